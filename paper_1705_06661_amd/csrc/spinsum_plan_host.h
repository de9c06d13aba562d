// spinsum_plan_host.h -- host-side plan object of libspinsum (internal).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/spinsum.h"
#include "spinsum_internal.h"

namespace spinsum {

// The symmetric group S_d with its elements in lexicographic order.
struct SymGroup {
  int d = 0;
  int df = 0;
  std::vector<std::vector<int>> p;  // p[r] = the r-th permutation
  std::vector<int> inv;             // rank of the inverse
  std::vector<int> mul;             // mul[a*df+b] = rank of "a after b": m -> a[b[m]]
  void init(int d);
  int rank(const int* q) const;
};

// One tile orbit {sigma . B} of the block grid of a cube (host tables).
struct OrbitHost {
  int ntiles = 0;
  int ragged = 0;
  int B[kMaxD] = {0, 0, 0, 0};        // sorted block tuple
  int32_t tile_off[kMaxDF] = {};      // element offset of each tile origin
  int32_t tile_ext[kMaxDF] = {};      // packed extents of each tile
  int slot[kMaxDF] = {};              // tile of sigma . B, sigma in lex order
  int rep_off = 0, rep_cnt = 0;       // representatives in the pool
};

// Tables of one tensor (or one block of a batch) for one tile choice.
struct Tiling {
  Geom g{};
  int nb = 0;
  int vw = 1;
  int max_tiles = 0;        // tiles of the largest work item (group)
  int max_orbit_tiles = 0;  // tiles of the largest tile orbit
  int ragged = 0;
  int fits = 1;
  int64_t lds_elems = 0;
  int64_t nitems = 0;
  int chunks_per_thread = 0;  // 16-byte loads per thread for the largest item
  int max_rep_cnt = 0;        // representatives of the largest work item
  int nts = 1;                // non-temporal stores
  int ntl = 0;                // non-temporal tile loads (items own whole lines)
  std::vector<OrbitHost> orbits;
  std::vector<GroupDev> groups;
  std::vector<uint32_t> reps;
  // The same lists in lexicographic order where reps holds them in the
  // bank-spreading order (empty when no list was reordered).  Packing writes
  // one packed value per representative, and in this order the lanes of a
  // wave write neighbouring packed entries.
  std::vector<uint32_t> reps_lex;
};

}  // namespace spinsum

struct spinsum_plan_s {
  // problem
  int d = 0, n = 0;
  int group_first = 0;
  // The plan of the subgroup's axes (see reduce_to_moved_axes), which exec,
  // adjoint, set_tile, autotune and check_ownership use when it is set;
  // this plan keeps the tables of the whole group (coefficient gradients).
  spinsum_plan_s* sub = nullptr;
  int sub_first = 0;  // group position of the sub-plan's first axis
  int inner = 1;  // elements of the inner spectators (dims after the group)
  int ndim = 0;
  std::vector<int64_t> extents;
  int64_t ncubes = 0, elems = 0;
  int dtype = 0, inplace = 0;
  unsigned flags = 0;
  spinsum::SymGroup G;
  std::vector<std::vector<double>> stage_a;  // per stage: coefficient of each permutation rank
  std::vector<double> expanded;              // coefficient of each permutation rank
  std::vector<double> M, MT;                 // coefficient vectors (forward, adjoint), df each
  std::vector<double> SM, SMT;               // per-stage coefficient vectors, application order
  // zero coefficients (bit s: stage s in application order; expanded: the
  // pre-multiplied vector), see set_terms
  uint32_t sparse_expanded = 0, sparse_fwd = 0, sparse_adj = 0;

  // tiling (single tensor)
  spinsum_tile_t tile{};
  spinsum::Tiling T;
  // the coefficient gradient's own tiling where it differs from T: it holds
  // two tensors in LDS, so fewer of its workgroups fit a CU and it packs
  // consecutive orbits into items even where T does not (cg_pack)
  spinsum::Tiling Tc;
  bool cg_pack = false;
  // the coefficient gradient runs k_cgrad_split on the plan's own tiling:
  // tiled items of one tile orbit in the direct-LDS layout, at most
  // kCgSplitTiles tiles and kCgSplitUnits element orbits per thread, every
  // tile's chunks in one pass of the workgroup, no inner runs, d <= 3
  // (decided with the tables, upload_tables)
  bool cg_split = false;
  // unpacking's own tiling where it differs from T (pk_own): the largest
  // items that fit a CU (see build_unpack_tiling), with their workgroup size
  spinsum::Tiling Tu;
  bool pk_own = false;
  int pk_threads = 256;
  // Tu's items run persistently (k_unpack_persist), pk_persist_blocks
  // workgroups per CU (cache_occupancy)
  bool pk_persist = false;
  int pk_persist_blocks = 1;

  // index-pair form (SPINSUM_FLAG_INDEX_PAIRS): T.g describes one pair
  // block, T.reps holds the representative pool, T.nb / T.vw / T.ragged /
  // T.max_tiles / T.max_rep_cnt / T.lds_elems / T.nitems as for tile orbits
  bool pair = false;
  int pv = 0;                             // partner extent V
  spinsum::PairGeom pg{};
  std::vector<uint64_t> pair_orbits;      // sorted combined blocks per tile orbit

  // batch
  bool batched = false;
  int nblocks = 1;
  std::vector<spinsum::Tiling> btil;
  std::vector<spinsum::BatchBlock> blocks;
  std::vector<spinsum::BatchItem> items;
  std::vector<int64_t> block_elems;
  int batch_vw = 1;
  int64_t batch_lds_elems = 0;
  int64_t batch_rep_bytes = 0;  // LDS behind the tiles: representative lists / tile table
  int batch_grid = 0;
  std::vector<int> bns;          // group extent of each block
  std::vector<int64_t> bcs;      // spectator cubes of each block
  std::vector<int> brs;          // inner spectator run of each block (1: trailing group)
  int64_t batch_item_bytes = 0;  // whole-cube items are packed up to this size
  int batch_persistent = 0;      // 1: persistent workgroups walk the item list

  // device
  bool has_dev = false;
  int device = -1;
  int num_cus = 256;
  int lds_limit = spinsum::kMaxLdsBytes;
  void* d_orbits = nullptr;
  void* d_reps = nullptr;
  void* d_reps_lex = nullptr;  // Tiling::reps_lex on the device, if any
  void* d_mats = nullptr;   // M | MT | SM | SMT in the storage type
  void* d_blocks = nullptr;
  void* d_items = nullptr;
  void* d_grad_part = nullptr;  // kGradSlots x d! doubles (spinsum_coef_grad)
  void* d_cg_orbits = nullptr;  // Tc.groups, Tc.reps (cg_pack)
  void* d_cg_reps = nullptr;
  void* d_pk_orbits = nullptr;  // Tu.groups, Tu.reps (pk_own)
  void* d_pk_reps = nullptr;
  int last_hip_error = 0;
  int occ_blocks = 1;  // workgroups per CU of the persistent exec kernel (cache_occupancy)
  std::string why;
};

namespace spinsum {
// Implemented in spinsum_plan.cpp
spinsum_status build_tiling(const spinsum_plan_s& P, int n, int64_t ncubes,
                            const spinsum_tile_t& tile, int vw, Tiling* out);
// single: a single-tensor plan (may pick a packed two-blocks-per-axis tile)
spinsum_status choose_tile(const spinsum_plan_s& P, int n, int64_t ncubes, int vw,
                           spinsum_tile_t* tile, bool single);
int max_vector_width(const spinsum_plan_s& P, int64_t row);
spinsum_status upload_tables(spinsum_plan_s* P);

spinsum_status build_batched(spinsum_plan_s* P, int64_t item_bytes);
void free_device(spinsum_plan_s* P);
int elem_size(const spinsum_plan_s& P);
// Implemented in spinsum_exec.hip
spinsum_status cache_occupancy(spinsum_plan_s* P);
// Implemented in spinsum_tune.cpp
bool cache_lookup(const spinsum_plan_s& P, spinsum_tile_t* tile);
bool batched_cache_lookup(const spinsum_plan_s& P, int64_t* item_bytes, int* persistent);
}  // namespace spinsum
