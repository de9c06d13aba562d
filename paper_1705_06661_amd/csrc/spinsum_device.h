// spinsum_device.h -- gfx950 kernels of libspinsum (instantiated per storage
// type and group size in spinsum_kern_<type>_d<d>.hip).
//
// A work item is a run of whole spectator cubes, or one tile orbit
// {sigma . B} of one cube (the macro-kernel of Alg. 5b/6), optionally
// several tile orbits of a cube.  A workgroup
//   1. loads every tile of the item from HBM once, in 16-byte chunks along
//      the fastest (stride-one) axis, into LDS;
//   2. combines every element orbit: each thread takes representatives x,
//      reads v_sigma = tile[sigma . x] for all sigma in S_d, forms
//      w_tau = sum_sigma a(tau^-1 o sigma) v_sigma (a = the coefficient of
//      each permutation in the operator, in scalar registers; with stage
//      chaining the stages are applied one after the other) and writes w_tau
//      to tile[tau . x];
//   3. stores the tiles back once with 16-byte stores, non-temporal where
//      the planner chooses them (Sec. 4.6.3), in place (Sec. 4.6.5) or to
//      the output.
// With inner spectators every group position is a run of `inner` elements:
// tile rows are bl * inner elements long and the combine step runs over
// (representative, inner index) pairs.
// Every element belongs to exactly one item, and inside an item to the
// element orbit of exactly one representative, so in-place needs only the
// workgroup barriers.
//
// Kernels:
//   k_lds     one item per workgroup, loads straight into LDS
//             (global_load_lds), 256/512/1024 threads -- the default;
//   k_ldsp    persistent, two LDS buffers, next item's loads in flight;
//   k_exec    one item per workgroup, loads through registers into padded
//             LDS (rows that are not whole 16-byte chunks);
//   k_pipe    persistent, next item prefetched into registers;
//   k_batched many tensors, one item of the cost-sorted list per workgroup;
//   k_pair    index-pair form: one tile orbit of combined (partner, group)
//             blocks per workgroup, its tile list built in the workgroup;
//   k_cgrad   coefficient gradient (x and the upstream gradient in LDS).
// One-shot grids are XCD-grouped: the workgroups of XCD x (blockIdx % 8 == x)
// take a contiguous range of items, so the tile orbits of one cube -- which
// share cache lines along the fastest axis -- meet in the same L2.  The work
// is HBM-bound (0.75 flop/byte in 3D, 3 in 4D): no matrix cores are used.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "spinsum_plan_host.h"

namespace spinsum {
namespace {

constexpr int kThreads = 256;     // workgroup size of every kernel but k_lds
constexpr int kMaxThreads = 1024; // k_lds, k_ldsp: 256, 512 or 1024 (blockDim.x)
constexpr int kUnroll = 4;
constexpr int kUnpackBatch = 4;   // k_unpack: packed values requested together per thread

template <int D>
struct Fact {
  static constexpr int v = D * Fact<D - 1>::v;
};
template <>
struct Fact<0> {
  static constexpr int v = 1;
};

template <typename T, int VW>
struct VecT;
template <>
struct VecT<double, 1> {
  typedef double type;
};
template <>
struct VecT<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct VecT<float, 1> {
  typedef float type;
};
template <>
struct VecT<float, 2> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct VecT<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
};

template <typename V, typename T, int VW>
__device__ __forceinline__ T vget(const V& v, int k) {
  if constexpr (VW == 1)
    return v;
  else
    return v[k];
}
template <typename V, typename T, int VW>
__device__ __forceinline__ void vset(V& v, int k, T x) {
  if constexpr (VW == 1)
    v = x;
  else
    v[k] = x;
}

// Uniform tables (orbit descriptors, coefficients, batch items) are read
// through the constant address space: the compiler then uses scalar loads,
// which neither take vector registers nor wait behind the in-flight tile
// prefetch (vector-memory loads complete in order).
template <typename X>
using cptr = const __attribute__((address_space(4))) X*;

template <typename X>
__device__ __forceinline__ cptr<X> as_const(const X* p) {
  return (cptr<X>)(p);
}

__device__ __forceinline__ FastDiv load_fd(const __attribute__((address_space(4))) FastDiv& f) {
  FastDiv r;
  r.div = f.div;
  r.mul = f.mul;
  r.shift = f.shift;
  r.pad = 0;
  return r;
}

__device__ __forceinline__ Geom load_geom(const __attribute__((address_space(4))) Geom& s) {
  Geom g;
  g.cube_elems = s.cube_elems;
  g.ncubes = s.ncubes;
  g.n = s.n;
  g.bl = s.bl;
  g.ngroups = s.ngroups;
  g.cpw = s.cpw;
#pragma unroll
  for (int m = 0; m < kMaxD; ++m) {
    g.gst[m] = s.gst[m];
    g.lst[m] = s.lst[m];
  }
  g.ts = s.ts;
  g.cube_lds = s.cube_lds;
  g.rows = s.rows;
  g.vpr = s.vpr;
  g.inner = s.inner;
  g.pad0 = 0;
  g.fd_inner = load_fd(s.fd_inner);
  g.fd_vpr = load_fd(s.fd_vpr);
  g.fd_rows = load_fd(s.fd_rows);
  g.fd_bl = load_fd(s.fd_bl);
  g.fd_ngroups = load_fd(s.fd_ngroups);
  return g;
}

template <typename T>
struct ExecArgs {
  const T* in;
  T* out;
  const GroupDev* orbits;  // work-item templates (groups of tile orbits)
  const uint32_t* reps;
  const T* coef;    // coefficient vector(s), d! per stage
  Geom g;
  int64_t nitems;
  int64_t xcd_per;  // > 0: items grouped per XCD (items per XCD range)
  int32_t nstages;  // stages applied one after the other (chain mode)
  int32_t reverse;
  int32_t lds_tile_bytes;  // k_pipe: start of the representative copy in LDS;
                           // k_ldsp: bytes of one tile buffer
  int32_t nreps;           // k_ldsp: entries of the shared representative table
  uint32_t sparse;         // bit s: stage s has a zero coefficient (see combine_orbit)
  int32_t nt_loads;        // k_lds: non-temporal tile loads (items own whole lines)
};

template <typename T>
struct CGradArgs {
  const T* x;
  const T* gr;             // upstream gradient
  double* grad;            // kGradSlots x d! partial sums, lexicographic permutation order
  const GroupDev* orbits;
  const uint32_t* reps;
  Geom g;
  int64_t nitems;
  int64_t xcd_per;
  int32_t lds_tile_bytes;  // one tile region (x or gr)
  int32_t pad;
};

template <typename T>
struct BatchArgs {
  const T* const* in;
  T* const* out;
  const GroupDev* orbits;  // work-item templates (groups of tile orbits)
  const uint32_t* reps;
  const T* coef;
  const BatchBlock* blocks;
  const BatchItem* items;
  int64_t nitems;
  int64_t xcd_per;         // > 0: items grouped per XCD (items per XCD range)
  int32_t lds_tile_bytes;  // start of the representative lists in LDS
  uint32_t sparse;         // the operator has a zero coefficient (see combine_orbit)
};

template <typename T>
struct PairArgs {
  const T* in;
  T* out;
  const uint64_t* orbits;  // sorted combined blocks of each tile orbit, 16 bits each
  const uint32_t* reps;    // representative pool (lists selected by pair_key)
  const T* coef;
  Geom g;
  PairGeom pg;
  int64_t nitems;
  int64_t xcd_per;
  int32_t nstages;
  int32_t reverse;
  int32_t lds_tile_bytes;  // start of the representative list in LDS
  uint32_t sparse;         // bit s: stage s has a zero coefficient (see combine_orbit)
};

// Unpacking and packing: the packed tensor holds one value per strictly
// increasing tuple of group indices, in lexicographic order, per outer
// spectator index: [outer.., ncomb = C(N, d), inner..].
template <typename T>
struct PackArgs {
  const T* full_in;    // k_pack: the full tensor
  T* full_out;         // k_unpack: the full tensor
  const T* packed_in;  // k_unpack
  T* packed_out;       // k_pack
  const GroupDev* orbits;
  const uint32_t* reps;
  const T* coef;       // the operator's d! coefficients (forward vector)
  Geom g;
  int64_t nitems;
  int64_t xcd_per;
  int64_t ncomb;
  int32_t lds_tile_bytes;
  int32_t ntmpl;                         // k_unpack_persist: item templates
  int32_t tmpl_wg[kUnpackTemplates + 1];  // k_unpack_persist: first workgroup of each
};

// Fused multiply-add in the storage type (a float FMA for float: the
// generic builtin would promote to double).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// w_tau = sum_sigma a(tau^-1 o sigma) v_sigma, sigma in lexicographic
// order, every index a compile-time constant
template <typename T, int D, int TAU, int... S>
__device__ __forceinline__ T orbit_row(const T* a, const T* v, std::integer_sequence<int, S...>) {
  T acc = T(0);
  ((acc = fma_t(a[GinvMul<D, TAU, S>::value], v[S], acc)), ...);
  return acc;
}

template <typename T, int D, int... TAU>
__device__ __forceinline__ void orbit_rows(const T* a, const T* v, T* w,
                                           std::integer_sequence<int, TAU...>) {
  ((w[TAU] = orbit_row<T, D, TAU>(a, v, std::make_integer_sequence<int, Fact<D>::v>{})), ...);
}

// w = one stage's coefficient product of an element orbit (chained
// stages).
template <typename T, int D>
__device__ __forceinline__ void orbit_product(const T (&a)[Fact<D>::v], const T (&v)[Fact<D>::v],
                                              T (&w)[Fact<D>::v]) {
  orbit_rows<T, D>(a, v, w, std::make_integer_sequence<int, Fact<D>::v>{});
}

// The same product, each w_tau written to LDS as soon as it is formed (all
// v_sigma are already in registers, so the in-place writes are safe); only
// a few accumulators are live at a time.  (One FMA chain per row is fine:
// a wave64 FMA occupies its SIMD for four cycles, which covers the
// dependency latency.)
template <typename T, int D, int... TAU>
__device__ __forceinline__ void orbit_rows_store_tail(const T* a, const T* v, T* lds, const int* addr,
                                                      std::integer_sequence<int, TAU...>) {
  ((lds[addr[TAU + 1]] =
        orbit_row<T, D, TAU + 1>(a, v, std::make_integer_sequence<int, Fact<D>::v>{})),
   ...);
}

// Combine one element orbit in place in LDS (pre-multiplied operator).
// Returns w_0, which tells whether an input was Inf or NaN: w_0 is formed
// over every sigma, zero coefficients included, so one Inf or NaN among the
// v_sigma makes it Inf or NaN (a * Inf is +-Inf, 0 * Inf and anything with
// NaN are NaN, and a sum holding a non-finite term stays non-finite); a
// finite w_0 means every input was finite and the dense product was exact.
template <typename T, int D>
__device__ __forceinline__ T orbit_store(const T (&a)[Fact<D>::v], const T (&v)[Fact<D>::v],
                                         T* lds, const int (&addr)[Fact<D>::v]) {
  constexpr int DF = Fact<D>::v;
  const T w0 = orbit_row<T, D, 0>(a, v, std::make_integer_sequence<int, DF>{});
  lds[addr[0]] = w0;
  orbit_rows_store_tail<T, D>(a, v, lds, addr, std::make_integer_sequence<int, DF - 1>{});
  return w0;
}

// Unit i of an orbit's combine loop -> cube of the item ci, representative
// ri and inner spectator index s: units run over (cube, representative,
// inner index) with the inner index fastest, so that the lanes of a wave
// read neighbouring LDS words when inner > 1.
__device__ __forceinline__ void split_unit(const Geom& g, uint32_t i, uint32_t rep_cnt,
                                           const FastDiv& fdr, int ncub, uint32_t* ci,
                                           uint32_t* ri, uint32_t* s) {
  uint32_t j = i;
  *s = 0;
  if (g.inner != 1) {
    j = fdiv(i, g.fd_inner);
    *s = i - j * (uint32_t)g.inner;
  }
  *ci = (ncub == 1) ? 0u : fdiv(j, fdr);
  *ri = j - *ci * rep_cnt;
}

// Combine the element orbits of one tile orbit: sb[sigma] = LDS offset of
// tile sigma . B, rp = its representative list (rep_cnt entries, local
// coordinates packed one byte per axis), for ncub cubes of the item.
// Returns (per thread) whether one of its element orbits had an Inf or NaN
// input (see orbit_store; with chained stages the last stage's w_0 tells,
// since a non-finite value reaches every row of every later stage).  Where
// the operator leaves out a permutation, such an item is redone by
// redo_orbit, kept out of this loop so that the dense product's registers
// stay as they are.
template <typename T, int D, bool CHAIN>
__device__ __forceinline__ bool combine_orbit(const Geom& g, const int32_t (&sb)[Fact<D>::v],
                                              const uint32_t* rp, uint32_t rep_cnt,
                                              const FastDiv& fdr, int ncub, cptr<T> coef,
                                              int nstages, T (&a)[Fact<D>::v], T* lds) {
  constexpr int DF = Fact<D>::v;
  const uint32_t nrep = (uint32_t)ncub * rep_cnt * (uint32_t)g.inner;
  bool bad = false;
  for (uint32_t i = threadIdx.x; i < nrep; i += blockDim.x) {
    uint32_t ci, ri, si;
    split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
    uint32_t pk = rp[ri];
    int l[D];
#pragma unroll
    for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
    const int base = (int)ci * g.cube_lds + (int)si;
    int addr[DF];
    T v[DF];
    orbit_addrs<D>(g, base, sb, l, addr, std::make_integer_sequence<int, DF>{});
#pragma unroll
    for (int r = 0; r < DF; ++r) v[r] = lds[addr[r]];
    if constexpr (!CHAIN) {
      const T w0 = orbit_store<T, D>(a, v, lds, addr);
      bad |= !__builtin_isfinite(w0);
    } else {
      T w[DF];
      for (int s = 0; s < nstages; ++s) {
#pragma unroll
        for (int r = 0; r < DF; ++r) a[r] = coef[s * DF + r];
        orbit_product<T, D>(a, v, w);
#pragma unroll
        for (int r = 0; r < DF; ++r) v[r] = w[r];
      }
      bad |= !__builtin_isfinite(v[0]);
#pragma unroll
      for (int r = 0; r < DF; ++r) lds[addr[r]] = v[r];
    }
  }
  return bad;
}

// 2. combine every element orbit of the item in LDS
// Combine every element orbit of a work item.  The item's tile orbits are
// visited in turn (uniform loop); their representatives come from global
// memory (REPS_IN_LDS false: reps + rep_off[k]) or from the item's LDS copy
// (true: reps + rep_base[k]).  Returns the per-thread flag of combine_orbit.
template <typename T, int D, bool CHAIN, bool REPS_IN_LDS>
__device__ __forceinline__ bool combine_item(const Geom& g, cptr<GroupDev> gd,
                                             const uint32_t* reps, cptr<T> coef, int nstages,
                                             int ncub, T* lds) {
  constexpr int DF = Fact<D>::v;
  T a[DF];
  if constexpr (!CHAIN) {
#pragma unroll
    for (int r = 0; r < DF; ++r) a[r] = coef[r];
  }
  bool bad = false;
  const int norb = gd->norb;
  for (int k = 0; k < norb; ++k) {
    int32_t sb[DF];
#pragma unroll
    for (int r = 0; r < DF; ++r) sb[r] = gd->slot_base[k][r];
    const FastDiv fdr = load_fd(gd->fd_rep[k]);
    const uint32_t* rp = reps + (REPS_IN_LDS ? gd->rep_base[k] : gd->rep_off[k]);
    bad |= combine_orbit<T, D, CHAIN>(g, sb, rp, (uint32_t)gd->rep_cnt[k], fdr, ncub, coef, nstages,
                                      a, lds);
  }
  return bad;
}

// Tables of S_d for (wave-uniform) runtime indices, read by the 4D redo: the
// rank of tau^-1 o sigma, and the inverse of the r-th permutation
// (inv[r][j] = m where lex_perm(r, m) = j).  The unrolled dense product
// takes the same values as template constants.
template <int D>
struct RuntimeTables {
  int8_t ginv[Fact<D>::v * Fact<D>::v];
  int8_t inv[Fact<D>::v][kMaxD];
  constexpr RuntimeTables() : ginv(), inv() {
    for (int t = 0; t < Fact<D>::v; ++t)
      for (int s = 0; s < Fact<D>::v; ++s) ginv[t * Fact<D>::v + s] = (int8_t)ginv_mul(D, t, s);
    for (int r = 0; r < Fact<D>::v; ++r)
      for (int m = 0; m < D; ++m) inv[r][lex_perm(D, r, m)] = (int8_t)m;
  }
};
template <int D>
__constant__ const RuntimeTables<D> kRuntimeTables = RuntimeTables<D>();

// Strides of group axis m (wave-uniform runtime m < D): in LDS and in the
// tensor.
__device__ __forceinline__ int32_t lds_stride(const Geom& g, int m) {
  return m == 0 ? g.lst[0] : m == 1 ? g.lst[1] : m == 2 ? g.lst[2] : g.lst[3];
}
__device__ __forceinline__ int32_t glb_stride(const Geom& g, int m) {
  return m == 0 ? g.gst[0] : m == 1 ? g.gst[1] : m == 2 ? g.gst[2] : g.gst[3];
}

// The element orbits of one tile orbit again, over the operator's own terms
// only: a permutation whose coefficient is zero is not a term of the sum
// (Def. 3), so its input is not read, and an Inf or NaN input reaches only
// the outputs of the terms that read it (the dense product, exact for
// finite inputs, would also give 0 * Inf = NaN elsewhere).  This runs only
// for items in which combine_orbit saw a non-finite input.  The inputs are
// read from the tensor `gin` (the item's cube), which still holds them: the
// item's stores come later, and no other workgroup writes its elements.
// Every output is formed over the nonzero coefficients in the dense
// product's order, so both forms below give the term-by-term sum bit for
// bit.  ltile(s) / gtile(s): LDS and tensor offset of tile sigma_s . B.

// Element offset of sigma_R . x inside its tile, for the strides st[] of
// the group axes (LDS or tensor).
template <int D, int R, int... M>
__device__ __forceinline__ int perm_offset(const int32_t* st, const int* l,
                                           std::integer_sequence<int, M...>) {
  return ((l[LexPerm<D, R, M>::value] * st[M]) + ... + 0);
}

// The d! inputs of an element orbit: each load takes its tile's origin as a
// wave-uniform base and a 32-bit offset inside the item (below 2^31: an
// item is at most cubes_per_wg cubes, which the planner keeps under 2 GiB).
template <typename T, int D, typename GT, int... R>
__device__ __forceinline__ void redo_gather(const Geom& g, GT gtile, const int* l, int gbase,
                                            const T* gin, T* v, std::integer_sequence<int, R...>) {
  ((v[R] = (gin + gtile(R))[gbase + perm_offset<D, R>(g.gst, l, std::make_integer_sequence<int, D>{})]),
   ...);
}

// w_tau over the operator's terms only: a zero coefficient reads nothing.
// The coefficients are read where they are used, from the constant address
// space (scalar loads), so that they take no vector registers.
template <typename T, int D, int TAU, int... S>
__device__ __forceinline__ T orbit_row_terms(cptr<T> a, const T* v, std::integer_sequence<int, S...>) {
  T acc = T(0);
  ((acc = (a[GinvMul<D, TAU, S>::value] != T(0)) ? fma_t(a[GinvMul<D, TAU, S>::value], v[S], acc)
                                                 : acc),
   ...);
  return acc;
}

template <typename T, int D, int... TAU>
__device__ __forceinline__ void orbit_rows_terms(cptr<T> a, const T* v, T* w,
                                                 std::integer_sequence<int, TAU...>) {
  ((w[TAU] = orbit_row_terms<T, D, TAU>(a, v, std::make_integer_sequence<int, Fact<D>::v>{})), ...);
}

template <typename T, int D, typename LT, int... TAU>
__device__ __forceinline__ void redo_store(const Geom& g, LT ltile, const int* l, int lbase,
                                           const T* w, T* lds, std::integer_sequence<int, TAU...>) {
  ((lds[lbase + ltile(TAU) + perm_offset<D, TAU>(g.lst, l, std::make_integer_sequence<int, D>{})] =
        w[TAU]),
   ...);
}

// Each w_tau formed and stored at once (one stage): no vector of results
template <typename T, int D, typename LT, int... TAU>
__device__ __forceinline__ void redo_rows_store(const Geom& g, LT ltile, const int* l, int lbase,
                                                cptr<T> a, const T* v, T* lds,
                                                std::integer_sequence<int, TAU...>) {
  ((lds[lbase + ltile(TAU) + perm_offset<D, TAU>(g.lst, l, std::make_integer_sequence<int, D>{})] =
        orbit_row_terms<T, D, TAU>(a, v, std::make_integer_sequence<int, Fact<D>::v>{})),
   ...);
}

// Each element orbit's d! inputs gathered into registers in one trip
// (addresses from compile-time permutation tables, as in the LDS gather),
// then the outputs formed from them.
template <typename T, int D, bool CHAIN, typename LT, typename GT>
__device__ __forceinline__ void redo_orbit_gather(const Geom& g, LT ltile, GT gtile, const uint32_t* rp,
                                           uint32_t rep_cnt, const FastDiv& fdr, int ncub,
                                           cptr<T> coef, int nstages, const T* gin, T* lds) {
  constexpr int DF = Fact<D>::v;
  const uint32_t nrep = (uint32_t)ncub * rep_cnt * (uint32_t)g.inner;
  for (uint32_t i = threadIdx.x; i < nrep; i += blockDim.x) {
    uint32_t ci, ri, si;
    split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
    const uint32_t pk = rp[ri];
    int l[D];
#pragma unroll
    for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
    const int lbase = (int)ci * g.cube_lds + (int)si;
    const int gbase = (int)ci * (int)g.cube_elems + (int)si;
    T v[DF];
    redo_gather<T, D>(g, gtile, l, gbase, gin, v, std::make_integer_sequence<int, DF>{});
    if constexpr (!CHAIN) {
      redo_rows_store<T, D>(g, ltile, l, lbase, coef, v, lds, std::make_integer_sequence<int, DF>{});
    } else {
      T w[DF];
      for (int st = 0; st < nstages; ++st) {
        orbit_rows_terms<T, D>(coef + st * DF, v, w, std::make_integer_sequence<int, DF>{});
#pragma unroll
        for (int r = 0; r < DF; ++r) v[r] = w[r];
      }
      redo_store<T, D>(g, ltile, l, lbase, v, lds, std::make_integer_sequence<int, DF>{});
    }
  }
}

// The terms walked in loops with few registers: coefficients and ranks from
// scalar loads, every address formed at run time, no register array
// indexed at run time.  One stage: the outputs in blocks of kRedoBlock,
// each input loaded once per block (d! / kRedoBlock times per element
// orbit instead of d! times).  Chained stages keep each element orbit's
// intermediate values in private memory.
constexpr int kRedoBlock = 8;

template <typename T, int D, bool CHAIN, typename LT, typename GT>
__device__ __forceinline__ void redo_orbit_loops(const Geom& g, LT ltile, GT gtile, const uint32_t* rp,
                                           uint32_t rep_cnt, const FastDiv& fdr, int ncub,
                                           cptr<T> coef, int nstages, const T* gin, T* lds) {
  constexpr int DF = Fact<D>::v;
  const RuntimeTables<D>& tb = kRuntimeTables<D>;
  const uint32_t nrep = (uint32_t)ncub * rep_cnt * (uint32_t)g.inner;
  for (uint32_t i = threadIdx.x; i < nrep; i += blockDim.x) {
    uint32_t ci, ri, si;
    split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
    const uint32_t pk = rp[ri];
    int l[D];
#pragma unroll
    for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
    const int lbase = (int)ci * g.cube_lds + (int)si;
    const int64_t gbase = (int64_t)ci * g.cube_elems + (int64_t)si;
    auto laddr = [&](int s) {
      int x = lbase + ltile(s);
#pragma unroll
      for (int j = 0; j < D; ++j) x += l[j] * lds_stride(g, tb.inv[s][j]);
      return x;
    };
    auto gaddr = [&](int s) {
      int64_t x = gbase + gtile(s);
#pragma unroll
      for (int j = 0; j < D; ++j) x += (int64_t)l[j] * glb_stride(g, tb.inv[s][j]);
      return x;
    };
    if constexpr (!CHAIN) {
      // kRedoBlock outputs at a time: each input is loaded once per block
      // and feeds that many accumulators
#pragma unroll 1
      for (int t0 = 0; t0 < DF; t0 += kRedoBlock) {
        T acc[kRedoBlock];
#pragma unroll
        for (int u = 0; u < kRedoBlock; ++u) acc[u] = T(0);
#pragma unroll 4
        for (int s = 0; s < DF; ++s) {
          const T x = gin[gaddr(s)];
#pragma unroll
          for (int u = 0; u < kRedoBlock; ++u) {
            const T c = coef[tb.ginv[(t0 + u) * DF + s]];
            acc[u] = (c != T(0)) ? fma_t(c, x, acc[u]) : acc[u];
          }
        }
#pragma unroll
        for (int u = 0; u < kRedoBlock; ++u) lds[laddr(t0 + u)] = acc[u];
      }
    } else {
      volatile T cur[DF];
      volatile T nxt[DF];
#pragma unroll 1
      for (int s = 0; s < DF; ++s) cur[s] = gin[gaddr(s)];
#pragma unroll 1
      for (int st = 0; st < nstages; ++st) {
#pragma unroll 1
        for (int t = 0; t < DF; ++t) {
          T acc = T(0);
#pragma unroll 1
          for (int s = 0; s < DF; ++s) {
            const T c = coef[st * DF + tb.ginv[t * DF + s]];
            if (c != T(0)) acc = fma_t(c, cur[s], acc);
          }
          nxt[t] = acc;
        }
#pragma unroll 1
        for (int t = 0; t < DF; ++t) cur[t] = nxt[t];
      }
#pragma unroll 1
      for (int t = 0; t < DF; ++t) lds[laddr(t)] = cur[t];
    }
  }
}

// d <= 3: gather each element orbit's inputs once (a few registers, short
// code).  d = 4: the gathered form (24 inputs, 576 guarded FMAs unrolled)
// made the dense path of the same kernels 2-5 % slower (registers and code
// size), so 4D walks the terms in loops that keep eight loads in flight.
template <typename T, int D, bool CHAIN, typename LT, typename GT>
__device__ __forceinline__ void redo_orbit(const Geom& g, LT ltile, GT gtile, const uint32_t* rp,
                                           uint32_t rep_cnt, const FastDiv& fdr, int ncub,
                                           cptr<T> coef, int nstages, const T* gin, T* lds) {
  if constexpr (D <= 3)
    redo_orbit_gather<T, D, CHAIN>(g, ltile, gtile, rp, rep_cnt, fdr, ncub, coef, nstages, gin, lds);
  else
    redo_orbit_loops<T, D, CHAIN>(g, ltile, gtile, rp, rep_cnt, fdr, ncub, coef, nstages, gin, lds);
}

// redo_orbit for every tile orbit of a work item (the GroupDev tables: tile
// sigma . B of orbit k sits at LDS offset slot_base[k][sigma], which is its
// slot times g.ts, and at tile_off[slot] in the cube).
template <typename T, int D, bool CHAIN, bool REPS_IN_LDS>
__device__ __forceinline__ void redo_item(const Geom& g, cptr<GroupDev> gd, const uint32_t* reps,
                                          cptr<T> coef, int nstages, int ncub, const T* gin,
                                          T* lds) {
  const int norb = gd->norb;
  const uint32_t ts = (uint32_t)g.ts;
  for (int k = 0; k < norb; ++k) {
    auto ltile = [&](int s) -> int32_t { return gd->slot_base[k][s]; };
    auto gtile = [&](int s) -> int64_t {
      return gd->tile_off[(uint32_t)gd->slot_base[k][s] / ts];
    };
    const FastDiv fdr = load_fd(gd->fd_rep[k]);
    const uint32_t* rp = reps + (REPS_IN_LDS ? gd->rep_base[k] : gd->rep_off[k]);
    redo_orbit<T, D, CHAIN>(g, ltile, gtile, rp, (uint32_t)gd->rep_cnt[k], fdr, ncub, coef, nstages,
                            gin, lds);
  }
}

// After the dense combine of an item: does the item have to be redone over
// the operator's own terms?  Only when the operator (or a chained stage)
// leaves out a permutation and some thread saw an Inf or NaN input.  The
// answer travels through one LDS word, cleared by clear_terms_flag before a
// barrier that precedes the combine, set by the first lane of every wave
// that saw one, and read after this function's barrier -- the workgroup
// barrier that the store phase needs anyway.
__shared__ uint32_t terms_flag;

__device__ __forceinline__ void clear_terms_flag(uint32_t sparse) {
  if (sparse != 0u && threadIdx.x == 0) terms_flag = 0u;
}

__device__ __forceinline__ bool item_needs_terms(uint32_t sparse, bool bad) {
  if (sparse != 0u && __builtin_amdgcn_ballot_w64(bad) != 0ull && (threadIdx.x & 63u) == 0u)
    __hip_atomic_fetch_or(&terms_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __syncthreads();
  return sparse != 0u && terms_flag != 0u;
}

__device__ __forceinline__ void stage_tinfo(int32_t* tinfo, const GroupDev* __restrict__ gd) {
  const int nt = gd->ntiles;
  if ((int)threadIdx.x < nt) {
    tinfo[threadIdx.x] = gd->tile_off[threadIdx.x];
    tinfo[kMaxDF + threadIdx.x] = gd->tile_ext[threadIdx.x];
  }
}

// 1a. issue the loads of an item into registers (no wait)
template <typename T, int D, int VW, int MAXC>
__device__ __forceinline__ void issue_loads(const Geom& g, const int32_t* tinfo, int ntiles,
                                            bool ragged, uint32_t nchunks, const T* sbase,
                                            typename VecT<T, VW>::type (&buf)[MAXC],
                                            int (&lo)[MAXC]) {
  typedef typename VecT<T, VW>::type V;
#pragma unroll
  for (int u = 0; u < MAXC; ++u) {
    uint32_t c = threadIdx.x + u * kThreads;
    int go = 0;
    int l = 0;
    bool ok = (c < nchunks) && chunk_addr<D, VW>(g, c, ntiles, tinfo, tinfo + kMaxDF, ragged, &go, &l);
    lo[u] = ok ? l : -1;
    if (ok) buf[u] = *reinterpret_cast<const V*>(sbase + go);
  }
}

// 1b. write the loaded registers to LDS (waits for the loads)
template <typename T, int VW, int MAXC>
__device__ __forceinline__ void fill_lds(const typename VecT<T, VW>::type (&buf)[MAXC],
                                         const int (&lo)[MAXC], T* lds) {
  typedef typename VecT<T, VW>::type V;
#pragma unroll
  for (int u = 0; u < MAXC; ++u)
    if (lo[u] >= 0) {
#pragma unroll
      for (int k = 0; k < VW; ++k) lds[lo[u] + k] = vget<V, T, VW>(buf[u], k);
    }
}

// 3. store every tile of the item
template <typename T, int D, int VW, bool NTS>
__device__ __forceinline__ void store_item(const Geom& g, const int32_t* tinfo, int ntiles,
                                           bool ragged, uint32_t nchunks, T* dbase,
                                           const T* lds) {
  typedef typename VecT<T, VW>::type V;
  for (uint32_t c0 = threadIdx.x; c0 < nchunks; c0 += kUnroll * kThreads) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint32_t c = c0 + u * kThreads;
      int go = 0;
      int lo = 0;
      bool ok = (c < nchunks) && chunk_addr<D, VW>(g, c, ntiles, tinfo, tinfo + kMaxDF, ragged, &go, &lo);
      if (ok) {
        V val;
#pragma unroll
        for (int k = 0; k < VW; ++k) vset<V, T, VW>(val, k, lds[lo + k]);
        V* p = reinterpret_cast<V*>(dbase + go);
        if constexpr (NTS)
          __builtin_nontemporal_store(val, p);
        else
          *p = val;
      }
    }
  }
}

// item index -> (first cube, orbit, cube count)
__device__ __forceinline__ void decode_item(const Geom& g, int64_t item, int64_t* cube0,
                                            int* orbit, int* ncub) {
  if (g.bl == g.n) {
    *cube0 = item * g.cpw;
    *orbit = 0;
    int64_t left = g.ncubes - *cube0;
    *ncub = (int)(left < g.cpw ? left : g.cpw);
  } else {
    uint32_t q = fdiv((uint32_t)item, g.fd_ngroups);
    *cube0 = q;
    *orbit = (int)((uint32_t)item - q * (uint32_t)g.ngroups);
    *ncub = 1;
  }
}

// One-shot: one item per workgroup.
template <typename T, int D, int VW, bool CHAIN, bool NTS>
__global__ void __launch_bounds__(kThreads) k_exec(const ExecArgs<T> a) {
  typedef typename VecT<T, VW>::type V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int32_t tinfo[2 * kMaxDF];
  T* lds = reinterpret_cast<T*>(smem);
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  if (a.reverse) item = a.nitems - 1 - item;
  const Geom& g = a.g;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, item, &cube0, &orbit, &ncub);
  const GroupDev* od = a.orbits + orbit;
  cptr<GroupDev> cod = as_const(od);
  clear_terms_flag(a.sparse);
  stage_tinfo(tinfo, od);
  __syncthreads();
  const int ntiles = cod->ntiles;
  const bool ragged = cod->ragged != 0;
  const uint32_t nchunks = (uint32_t)ncub * (uint32_t)ntiles * (uint32_t)g.rows * (uint32_t)g.vpr;
  const T* sbase = a.in + cube0 * g.cube_elems;
  for (uint32_t c0 = 0; c0 < nchunks; c0 += kUnroll * kThreads) {
    V buf[kUnroll];
    int lo[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint32_t c = c0 + threadIdx.x + u * kThreads;
      int go = 0;
      int l = 0;
      bool ok = (c < nchunks) && chunk_addr<D, VW>(g, c, ntiles, tinfo, tinfo + kMaxDF, ragged, &go, &l);
      lo[u] = ok ? l : -1;
      if (ok) buf[u] = *reinterpret_cast<const V*>(sbase + go);
    }
    fill_lds<T, VW, kUnroll>(buf, lo, lds);
  }
  __syncthreads();
  const bool bad =
      combine_item<T, D, CHAIN, false>(g, cod, a.reps, as_const(a.coef), a.nstages, ncub, lds);
  if (item_needs_terms(a.sparse, bad)) {
    redo_item<T, D, CHAIN, false>(g, cod, a.reps, as_const(a.coef), a.nstages, ncub, sbase, lds);
    __syncthreads();
  }
  store_item<T, D, VW, NTS>(g, tinfo, ntiles, ragged, nchunks, a.out + cube0 * g.cube_elems, lds);
}

// Chunk c (VW elements) of a full tile, chunks in row-major order: its
// local coordinates l (l[D-1] is the chunk's first element inside its row
// of bl * inner elements).
template <int D, int VW>
__device__ __forceinline__ void chunk_coords(const Geom& g, uint32_t c, int (&l)[D]) {
  uint32_t q = fdiv(c, g.fd_vpr);
  l[D - 1] = (int)(c - q * (uint32_t)g.vpr) * VW;
  if constexpr (D == 2) {
    l[0] = (int)q;
  } else {
    uint32_t r = q;
#pragma unroll
    for (int m = D - 2; m >= 1; --m) {
      uint32_t qq = fdiv(r, g.fd_bl);
      l[m] = (int)(r - qq * (uint32_t)g.bl);
      r = qq;
    }
    l[0] = (int)r;
  }
}

// Inside the extent of a ragged tile (ext packs one byte per index)?
template <int D>
__device__ __forceinline__ bool chunk_inside(const int (&l)[D], int ext, int inner) {
  bool in = true;
#pragma unroll
  for (int m = 0; m < D - 1; ++m) in = in && (l[m] < ((ext >> (8 * m)) & 255));
  return in && (l[D - 1] < ((ext >> (8 * (D - 1))) & 255) * inner);
}

// Element offset of a chunk inside its tile (the last coordinate counts
// elements of the row).
template <int D>
__device__ __forceinline__ int chunk_offset(const Geom& g, const int (&l)[D]) {
  int off = l[D - 1];
#pragma unroll
  for (int m = 0; m < D - 1; ++m) off += l[m] * g.gst[m];
  return off;
}

// One 16-byte direct-to-LDS load with the default cache policy, or with the
// non-temporal one (NTL: the NT bit, value 2, of the cache-policy operand;
// sc0 = 1 and sc1 = 16 measured no different from the default here).
// Non-temporal loads suit work items that own whole
// 128-byte lines -- tile rows of whole lines, or whole cubes copied as one
// run: nothing else reads those lines, so they need not stay in the L2
// (measured: +3 to +6 %).  Where tile rows fill parts of lines that other
// items read, the lines must stay for them, and the default policy is
// 14 to 28 % faster.
template <bool NTL>
__device__ __forceinline__ void load_lds16(const void* src, __attribute__((address_space(3))) void* dst) {
  if constexpr (NTL)
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 2);
  else
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

// Issue the loads of one item straight into LDS (global_load_lds_dwordx4:
// lane i of a wave writes 16 bytes at the wave's LDS base + 16 i).  LDS
// holds the tiles densely in chunk order: tile t at element t * ts, chunk c
// at c * VW.  A chunk has the same position in every tile, so its address
// arithmetic is done once and reused for all tiles of the item.  Returns,
// uniformly over the wave, how many load instructions this wave issued with
// at least one active lane -- a lower bound on the vector-memory operations
// the item added to the wave's vmcnt.
template <typename T, int D, bool NTL = false>
__device__ __forceinline__ int issue_item_lds(const Geom& g, cptr<GroupDev> od, bool whole,
                                              int ntl, bool ragged, const T* src,
                                              unsigned char* lds_bytes) {
  constexpr int VW = 16 / sizeof(T);
  const uint32_t cpt = (uint32_t)g.rows * (uint32_t)g.vpr;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave_bytes = (tid >> 6) * 1024u;
  int issued = 0;
  for (uint32_t c0 = 0; c0 < cpt; c0 += blockDim.x) {
    int l[D];
    chunk_coords<D, VW>(g, c0 + tid, l);
    const int off = chunk_offset<D>(g, l);
    const bool in = c0 + tid < cpt;
    for (int t = 0; t < ntl; ++t) {
      const int toff = whole ? t * (int)g.cube_elems : od->tile_off[t];
      const bool ok = in && (!ragged || chunk_inside<D>(l, od->tile_ext[t], g.inner));
      const uint32_t lbyte = (uint32_t)(t * g.ts + (int)c0 * VW) * (uint32_t)sizeof(T) + wave_bytes;
      if (ok)
        load_lds16<NTL>((const void*)(src + toff + off),
                        (__attribute__((address_space(3))) void*)(lds_bytes + lbyte));
      issued += (__builtin_amdgcn_ballot_w64(ok) != 0ull) ? 1 : 0;
    }
  }
  return __builtin_amdgcn_readfirstlane(issued);
}

// Whole-cube items are one contiguous run of m elements starting at src.
// It is copied into LDS as it lies in memory, shifted so that 16-byte
// chunks of memory land on 16-byte chunks of LDS: with p0 = src rounded
// down to 16 bytes, element src + e goes to LDS element shift + e, where
// shift = (src - p0) / sizeof(T).  Whole chunks inside the run go
// global->LDS directly (global_load_lds_dwordx4); the partial chunks at
// either end (fewer than 16 / sizeof(T) elements each) go through
// registers.  Nothing outside the run is read.  Returns shift.
template <typename T, bool NTL = false>
__device__ __forceinline__ int flat_issue(const T* src, uint32_t m, unsigned char* lds) {
  constexpr uint32_t E = 16 / sizeof(T);
  const uintptr_t p = (uintptr_t)src;
  const uintptr_t p0 = p & ~(uintptr_t)15;
  const uintptr_t pend = p + (uintptr_t)m * sizeof(T);
  uintptr_t pc = (p + 15) & ~(uintptr_t)15;
  if (pc > pend) pc = pend;
  const uint32_t nfull = (uint32_t)((pend - pc) >> 4);
  const uintptr_t pf = pc + ((uintptr_t)nfull << 4);
  const uint32_t head = (uint32_t)((pc - p) / sizeof(T));
  const uint32_t tail = (uint32_t)((pend - pf) / sizeof(T));
  const uint32_t shift = (uint32_t)((p - p0) / sizeof(T));
  const uint32_t tid = threadIdx.x;
  T* ldsT = reinterpret_cast<T*>(lds);
  // partial chunks through registers (at most E - 1 elements each)
  if (tid < head) ldsT[shift + tid] = src[tid];
  if (tid >= 32 && tid - 32 < tail) {
    const uint32_t e = (uint32_t)((pf - p) / sizeof(T)) + (tid - 32);
    ldsT[shift + e] = src[e];
  }
  (void)E;
  const uint32_t lds0 = (uint32_t)(pc - p0);
  const uint32_t wave_bytes = (tid >> 6) * 1024u;
  for (uint32_t c0 = 0; c0 < nfull; c0 += blockDim.x) {
    if (c0 + tid < nfull)
      load_lds16<NTL>((const void*)(pc + ((uintptr_t)(c0 + tid) << 4)),
                      (__attribute__((address_space(3))) void*)(lds + lds0 + c0 * 16u + wave_bytes));
  }
  return (int)shift;
}

template <typename T>
__device__ __forceinline__ int flat_shift(const T* p) {
  return (int)(((uintptr_t)p & 15u) / sizeof(T));
}

// Store a whole-cube item from its LDS copy, whose element 0 sits at LDS
// element in_shift (as flat_issue left it): whole 16-byte chunks with vector
// stores (non-temporal when NTS), the partial chunks at either end element
// by element.  If dst is aligned differently from the loaded source, every
// element is stored on its own.
template <typename T, bool NTS>
__device__ __forceinline__ void flat_store(T* dst, uint32_t m, const unsigned char* lds,
                                           int in_shift) {
  typedef typename VecT<T, 16 / sizeof(T)>::type V;
  if (flat_shift(dst) != in_shift) {
    const T* ldsT = reinterpret_cast<const T*>(lds) + in_shift;
    for (uint32_t e = threadIdx.x; e < m; e += blockDim.x) dst[e] = ldsT[e];
    return;
  }
  const uintptr_t p = (uintptr_t)dst;
  const uintptr_t p0 = p & ~(uintptr_t)15;
  const uintptr_t pend = p + (uintptr_t)m * sizeof(T);
  uintptr_t pc = (p + 15) & ~(uintptr_t)15;
  if (pc > pend) pc = pend;
  const uint32_t nfull = (uint32_t)((pend - pc) >> 4);
  const uintptr_t pf = pc + ((uintptr_t)nfull << 4);
  const uint32_t head = (uint32_t)((pc - p) / sizeof(T));
  const uint32_t tail = (uint32_t)((pend - pf) / sizeof(T));
  const uint32_t shift = (uint32_t)((p - p0) / sizeof(T));
  const uint32_t tid = threadIdx.x;
  const T* ldsT = reinterpret_cast<const T*>(lds);
  if (tid < head) dst[tid] = ldsT[shift + tid];
  if (tid >= 32 && tid - 32 < tail) {
    const uint32_t e = (uint32_t)((pf - p) / sizeof(T)) + (tid - 32);
    dst[e] = ldsT[shift + e];
  }
  const uint32_t lds0 = (uint32_t)(pc - p0);
  for (uint32_t c = tid; c < nfull; c += blockDim.x) {
    const V val = *reinterpret_cast<const V*>(lds + lds0 + c * 16u);
    V* q = reinterpret_cast<V*>(pc + ((uintptr_t)c << 4));
    if constexpr (NTS)
      __builtin_nontemporal_store(val, q);
    else
      *q = val;
  }
}

// Issue the loads of an item's representative lists straight into LDS
// (global_load_lds_dword: lane i of a wave writes 4 bytes at the wave's LDS
// base + 4 i): orbit k's list goes to rep_lds + rep_base[k].
__device__ __forceinline__ void issue_reps_lds(cptr<GroupDev> od, const uint32_t* reps,
                                               unsigned char* rep_lds) {
  const uint32_t tid = threadIdx.x;
  const uint32_t wave0 = tid & ~63u;
  const int norb = od->norb;
  for (int k = 0; k < norb; ++k) {
    const uint32_t cnt = (uint32_t)od->rep_cnt[k];
    const uint32_t* src = reps + od->rep_off[k];
    unsigned char* dst = rep_lds + (uint32_t)od->rep_base[k] * 4u;
    for (uint32_t i0 = 0; i0 < cnt; i0 += blockDim.x) {
      if (i0 + tid < cnt)
        __builtin_amdgcn_global_load_lds(
            (const void*)(src + i0 + tid),
            (__attribute__((address_space(3))) void*)(dst + (i0 + wave0) * 4u), 4, 0, 0);
    }
  }
}

// Store every tile of an item from its dense LDS copy (non-temporal when
// NTS).
template <typename T, int D, bool NTS>
__device__ __forceinline__ void store_item_lds(const Geom& g, cptr<GroupDev> od, bool whole,
                                               int ntl, bool ragged, T* dst, const T* lds) {
  constexpr int VW = 16 / sizeof(T);
  typedef typename VecT<T, VW>::type V;
  const uint32_t cpt = (uint32_t)g.rows * (uint32_t)g.vpr;
  for (uint32_t c0 = 0; c0 < cpt; c0 += blockDim.x) {
    const uint32_t c = c0 + threadIdx.x;
    int l[D];
    chunk_coords<D, VW>(g, c, l);
    const int off = chunk_offset<D>(g, l);
    const bool in = c < cpt;
    for (int t = 0; t < ntl; ++t) {
      const int toff = whole ? t * (int)g.cube_elems : od->tile_off[t];
      const bool ok = in && (!ragged || chunk_inside<D>(l, od->tile_ext[t], g.inner));
      if (ok) {
        const V val = *reinterpret_cast<const V*>(lds + t * g.ts + (int)c * VW);
        V* p = reinterpret_cast<V*>(dst + toff + off);
        if constexpr (NTS)
          __builtin_nontemporal_store(val, p);
        else
          *p = val;
      }
    }
  }
}

// Workgroup barrier for LDS written by ds_write only: wait for this wave's
// LDS operations (lgkmcnt(0), gfx9 encoding), then s_barrier; the signal
// fences keep the compiler from moving memory accesses across it.  A
// workgroup fence (__syncthreads) would also drain the vector memory
// counter, which holds the direct-to-LDS loads of the next item that are
// meant to stay in flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// s_waitcnt vmcnt(n) for a wave-uniform n: wait until at most n vector
// memory operations of this wave are outstanding (they complete in issue
// order).  Immediates in the gfx9 encoding (vmcnt in bits 3:0 and 15:14,
// expcnt and lgkmcnt left at their no-wait values); n above 31 waits for
// 31, which is stricter.
__device__ __forceinline__ void wait_vmcnt_atmost(int n) {
#define SPINSUM_VMCNT(N) \
  case N:                \
    __builtin_amdgcn_s_waitcnt(((N) & 15) | (0x7 << 4) | (0xF << 8) | (((N) >> 4) << 14)); \
    break;
  switch (n) {
    SPINSUM_VMCNT(0) SPINSUM_VMCNT(1) SPINSUM_VMCNT(2) SPINSUM_VMCNT(3)
    SPINSUM_VMCNT(4) SPINSUM_VMCNT(5) SPINSUM_VMCNT(6) SPINSUM_VMCNT(7)
    SPINSUM_VMCNT(8) SPINSUM_VMCNT(9) SPINSUM_VMCNT(10) SPINSUM_VMCNT(11)
    SPINSUM_VMCNT(12) SPINSUM_VMCNT(13) SPINSUM_VMCNT(14) SPINSUM_VMCNT(15)
    SPINSUM_VMCNT(16) SPINSUM_VMCNT(17) SPINSUM_VMCNT(18) SPINSUM_VMCNT(19)
    SPINSUM_VMCNT(20) SPINSUM_VMCNT(21) SPINSUM_VMCNT(22) SPINSUM_VMCNT(23)
    SPINSUM_VMCNT(24) SPINSUM_VMCNT(25) SPINSUM_VMCNT(26) SPINSUM_VMCNT(27)
    SPINSUM_VMCNT(28) SPINSUM_VMCNT(29) SPINSUM_VMCNT(30)
    default:
      __builtin_amdgcn_s_waitcnt((31 & 15) | (0x7 << 4) | (0xF << 8) | ((31 >> 4) << 14));
      break;
  }
#undef SPINSUM_VMCNT
}

// Wave priority (s_setprio) of the memory phases and of the combine step.
// A workgroup that is issuing its loads or stores runs ahead of the combine
// step of the other workgroups on its SIMD, so that the next loads leave
// the CU sooner; the combine step then fills the time the loads are in
// flight.  Measured: 4D 12^4 slab 4.80 -> 5.20 TB/s, 3D 32^3 slab
// unchanged (5.66 -> 5.70).
__device__ __forceinline__ void set_memory_priority() { __builtin_amdgcn_s_setprio(3); }
__device__ __forceinline__ void set_compute_priority() { __builtin_amdgcn_s_setprio(0); }

// One-shot with direct global->LDS loads (global_load_lds_dwordx4, 16 bytes
// per lane, no register staging): every load of the item is in flight at
// once.  LDS holds the tiles densely in chunk order -- tile t at t * ts,
// chunk c of a tile at c * VW -- which is the unpadded tile layout, so the
// planner builds this variant's tables with lds_pad = 0.  Tiles of a tile
// orbit, or the cubes of a whole-cube item, are visited with a uniform loop
// so that their base offsets come from scalar loads.  The item's
// representative lists are loaded into LDS behind the tiles in the same
// way, so the combine step issues no global loads.
// LDS: [tiles (lds_tile_bytes) | representatives (rep_total entries)].
template <typename T, int D, bool CHAIN, bool NTS>
__global__ void __launch_bounds__(kMaxThreads) k_lds(const ExecArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  if (a.reverse) item = a.nitems - 1 - item;
  const Geom& g = a.g;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, item, &cube0, &orbit, &ncub);
  const cptr<GroupDev> od = as_const(a.orbits + orbit);
  const bool whole = (g.bl == g.n);
  const int ntl = whole ? ncub : od->ntiles;
  const bool ragged = od->ragged != 0;
  // 1. tiles and representative lists straight into LDS, all in flight
  //    together
  unsigned char* rep_lds = smem + a.lds_tile_bytes;
  const uint32_t span = (uint32_t)ncub * (uint32_t)g.cube_elems;
  int shift = 0;
  clear_terms_flag(a.sparse);
  set_memory_priority();
  if (whole)
    shift = a.nt_loads ? flat_issue<T, true>(a.in + cube0 * g.cube_elems, span, smem)
                       : flat_issue<T, false>(a.in + cube0 * g.cube_elems, span, smem);
  else if (a.nt_loads)
    issue_item_lds<T, D, true>(g, od, whole, ntl, ragged, a.in + cube0 * g.cube_elems, smem);
  else
    issue_item_lds<T, D, false>(g, od, whole, ntl, ragged, a.in + cube0 * g.cube_elems, smem);
  issue_reps_lds(od, a.reps, rep_lds);
  set_compute_priority();
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): everything is in LDS
  __syncthreads();
  // 2. combine
  const bool bad = combine_item<T, D, CHAIN, true>(g, od, reinterpret_cast<const uint32_t*>(rep_lds),
                                                   as_const(a.coef), a.nstages, ncub, lds + shift);
  if (item_needs_terms(a.sparse, bad)) {
    redo_item<T, D, CHAIN, true>(g, od, reinterpret_cast<const uint32_t*>(rep_lds),
                                 as_const(a.coef), a.nstages, ncub, a.in + cube0 * g.cube_elems,
                                 lds + shift);
    __syncthreads();
  }
  // 3. store (the output may be shifted differently from the input)
  set_memory_priority();
  if (whole)
    flat_store<T, NTS>(a.out + cube0 * g.cube_elems, span, smem, shift);
  else
    store_item_lds<T, D, NTS>(g, od, whole, ntl, ragged, a.out + cube0 * g.cube_elems, lds);
}

// Index-pair form: one tile orbit {sigma . c} of one pair block per
// workgroup, c the orbit's sorted combined blocks (c_m = a_m * nb + b_m).
// Every wave forms the tile list itself: lane r forms sigma_r . c; tiles are
// numbered in the order of their first sigma, and slot r of the combine step
// is the tile of sigma_r . c.  Tiles then go straight into LDS: whole group
// cubes (bl == N) as one contiguous run each, with the run's 16-byte
// alignment shift folded into the slot offsets; otherwise in 16-byte chunks
// of rows, as in k_lds.
// LDS: [tiles (lds_tile_bytes) | representatives].

// Entry k of the unrolled permutation table: element m of permutation r
// (lexicographic) as a select chain, so that no register array is indexed
// with a lane-dependent value.
template <int D, int M, int... R>
__device__ __forceinline__ int perm_entry(int r, std::integer_sequence<int, R...>) {
  int v = 0;
  ((v = (r == R) ? LexPerm<D, R, M>::value : v), ...);
  return v;
}

// t = sigma_r . c for the packed tuple pk (16 bits per entry): entry m of
// the result is entry sigma_r[m] of c, taken with a variable shift (no
// register array indexed per lane).
template <int D, int... M>
__device__ __forceinline__ void permuted_tuple(uint64_t pk, int r, int (&t)[D],
                                               std::integer_sequence<int, M...>) {
  ((t[M] = (int)((pk >> (16 * perm_entry<D, M>(r, std::make_integer_sequence<int, Fact<D>::v>{}))) &
                 0xFFFFu)),
   ...);
}

template <typename T, int D, bool CHAIN, bool NTS>
__global__ void __launch_bounds__(kMaxThreads) k_pair(const PairArgs<T> a) {
  constexpr int DF = Fact<D>::v;
  constexpr int VW = 16 / sizeof(T);
  typedef typename VecT<T, VW>::type V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  if (a.reverse) item = a.nitems - 1 - item;
  const Geom& g = a.g;
  const PairGeom& pg = a.pg;
  const uint32_t q = fdiv((uint32_t)item, pg.fd_norb);
  const int64_t cube0 = q;
  const int64_t orb = item - (int64_t)q * pg.norb;
  const T* src = a.in + cube0 * g.cube_elems;
  T* dst = a.out + cube0 * g.cube_elems;
  // 1. the orbit's tile list, formed by every wave on its own (no barrier):
  //    lane r forms sigma_r . c, the distinct tiles are numbered in first-
  //    sigma order with a ballot, and lane t then holds tile t's origin,
  //    extents and alignment shift; the tile loops below take them with
  //    v_readlane (uniform index)
  const int lane = (int)(threadIdx.x & 63u);
  const uint64_t pk = as_const(a.orbits)[orb];
  int c[D];
#pragma unroll
  for (int m = 0; m < D; ++m) c[m] = (int)((pk >> (16 * m)) & 0xFFFFu);
  const bool act = lane < DF;
  int tt[D];
  permuted_tuple<D>(pk, act ? lane : 0, tt, std::make_integer_sequence<int, D>{});
  uint64_t key = 0;
#pragma unroll
  for (int m = 0; m < D; ++m) key |= (uint64_t)tt[m] << (16 * m);
  int first = lane;
  for (int r2 = DF - 1; r2 >= 0; --r2) {
    const uint64_t k2 = ((uint64_t)(uint32_t)__shfl((int)(key >> 32), r2, 64) << 32) |
                        (uint32_t)__shfl((int)(uint32_t)key, r2, 64);
    if (r2 < lane && k2 == key) first = r2;
  }
  const bool isfirst = act && first == lane;
  const uint64_t mask = __builtin_amdgcn_ballot_w64(isfirst);
  const int slot = __builtin_popcountll(mask & ((1ull << first) - 1ull));
  int64_t off = 0;
  int32_t ext = 0;
  int shift = 0;
  if (isfirst) {
    pair_tile(g, pg, D, tt, &off, &ext);
    if (pg.flat) shift = flat_shift<T>(src + off);
  }
  // LDS offset of tile sigma_r . c for lane r (the combine step's sb[r])
  const int sb_lane = slot * pg.tile_stride + __shfl(shift, act ? first : 0, 64);
  const int ntl = __builtin_popcountll(mask);
  int srcl = 0;  // the lane that formed tile `lane` (the lane-th set bit of mask)
  {
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < DF; ++r)
      if ((mask >> r) & 1ull) {
        if (cnt == lane) srcl = r;
        ++cnt;
      }
  }
  const int64_t my_toff =
      (int64_t)(((uint64_t)(uint32_t)__shfl((int)(off >> 32), srcl, 64) << 32) |
                (uint32_t)__shfl((int)(uint32_t)off, srcl, 64));
  const int32_t my_text = __shfl(ext, srcl, 64);
  const int my_shift = __shfl(shift, srcl, 64);
  uint32_t rep_cnt, rep_off;
  {
    const int k = pair_key(g, pg, D, c);
    rep_off = (uint32_t)pg.rep_off[k];
    rep_cnt = (uint32_t)pg.rep_cnt[k];
  }
  auto tile_off = [&](int t) -> int64_t {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)my_toff, t);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(my_toff >> 32), t);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };
  // 2. tiles and the representative list straight into LDS
  clear_terms_flag(a.sparse);
  set_memory_priority();
  const uint32_t tid = threadIdx.x;
  const uint32_t wave_bytes = (tid >> 6) * 1024u;
  const int64_t tile_elems = (int64_t)g.rows * g.bl * g.inner;
  auto issue_tiles = [&]() {
    if (pg.flat) {
      for (int t = 0; t < ntl; ++t) {
        const int64_t toff = tile_off(t);
        flat_issue<T, false>(src + toff, (uint32_t)tile_elems,
                      smem + (size_t)t * pg.tile_stride * sizeof(T));
      }
    } else {
      const uint32_t cpt = (uint32_t)g.rows * (uint32_t)g.vpr;
      for (uint32_t c0 = 0; c0 < cpt; c0 += blockDim.x) {
        int l[D];
        chunk_coords<D, VW>(g, c0 + tid, l);
        const int off = chunk_offset<D>(g, l);
        const bool in = c0 + tid < cpt;
        for (int t = 0; t < ntl; ++t) {
          const int64_t toff = tile_off(t);
          const bool ok = in && chunk_inside<D>(l, __builtin_amdgcn_readlane(my_text, t), g.inner);
          const uint32_t lbyte =
              (uint32_t)(t * pg.tile_stride + (int)c0 * VW) * (uint32_t)sizeof(T) + wave_bytes;
          if (ok)
            __builtin_amdgcn_global_load_lds(
                (const void*)(src + toff + off),
                (__attribute__((address_space(3))) void*)(smem + lbyte), 16, 0, 0);
        }
      }
    }
  };
  issue_tiles();
  unsigned char* rep_lds = smem + a.lds_tile_bytes;
  {
    const uint32_t wave0 = tid & ~63u;
    for (uint32_t i0 = 0; i0 < rep_cnt; i0 += blockDim.x)
      if (i0 + tid < rep_cnt)
        __builtin_amdgcn_global_load_lds(
            (const void*)(a.reps + rep_off + i0 + tid),
            (__attribute__((address_space(3))) void*)(rep_lds + (i0 + wave0) * 4u), 4, 0, 0);
  }
  set_compute_priority();
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): everything is in LDS
  __syncthreads();
  // 3. combine
  {
    T co[DF];
    const cptr<T> coef = as_const(a.coef);
    if constexpr (!CHAIN) {
#pragma unroll
      for (int r = 0; r < DF; ++r) co[r] = coef[r];
    }
    int32_t sb[DF];
#pragma unroll
    for (int r = 0; r < DF; ++r) sb[r] = __builtin_amdgcn_readlane(sb_lane, r);
    const FastDiv one{1u, 0u, 0u, 0u};
    const uint32_t* rp = reinterpret_cast<const uint32_t*>(rep_lds);
    const bool bad = combine_orbit<T, D, CHAIN>(g, sb, rp, rep_cnt, one, 1, coef,
                                                       a.nstages, co, lds);
    if (item_needs_terms(a.sparse, bad)) {
      // tile sigma_s . c: LDS slot sb[s] (its slot times the slot stride,
      // plus the slot's alignment shift, which is below the stride), at
      // tensor offset tile_off(slot)
      auto ltile = [&](int r) -> int32_t { return __builtin_amdgcn_readlane(sb_lane, r); };
      auto gtile = [&](int r) -> int64_t {
        return tile_off(__builtin_amdgcn_readlane(sb_lane, r) / pg.tile_stride);
      };
      redo_orbit<T, D, CHAIN>(g, ltile, gtile, rp, rep_cnt, one, 1, coef, a.nstages, src, lds);
      __syncthreads();
    }
  }
  // 4. store
  set_memory_priority();
  if (pg.flat) {
    for (int t = 0; t < ntl; ++t) {
      const int64_t toff = tile_off(t);
      flat_store<T, NTS>(dst + toff, (uint32_t)tile_elems,
                         smem + (size_t)t * pg.tile_stride * sizeof(T),
                         __builtin_amdgcn_readlane(my_shift, t));
    }
  } else {
    const uint32_t cpt = (uint32_t)g.rows * (uint32_t)g.vpr;
    for (uint32_t c0 = 0; c0 < cpt; c0 += blockDim.x) {
      const uint32_t c = c0 + tid;
      int l[D];
      chunk_coords<D, VW>(g, c, l);
      const int off = chunk_offset<D>(g, l);
      const bool in = c < cpt;
      for (int t = 0; t < ntl; ++t) {
        const int64_t toff = tile_off(t);
        const bool ok = in && chunk_inside<D>(l, __builtin_amdgcn_readlane(my_text, t), g.inner);
        if (ok) {
          const V val = *reinterpret_cast<const V*>(lds + t * pg.tile_stride + (int)c * VW);
          V* p = reinterpret_cast<V*>(dst + toff + off);
          if constexpr (NTS)
            __builtin_nontemporal_store(val, p);
          else
            *p = val;
        }
      }
    }
  }
}

// Persistent, double-buffered direct-LDS loads: while item k is combined
// and stored from one LDS buffer, the loads of item k+1 fill the other.
// The representative table of every orbit pattern is copied to LDS once.
// gridDim.x is a multiple of 8; workgroup j of XCD x walks the items of
// that XCD's contiguous range with stride gridDim.x / 8, so that the
// workgroups of one XCD work on neighbouring items at any time.
// LDS: [representatives (nreps, padded to 16 bytes) | buffer 0 | buffer 1].
template <typename T, int D, bool CHAIN, bool NTS>
__global__ void __launch_bounds__(kMaxThreads) k_ldsp(const ExecArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const Geom& g = a.g;
  uint32_t* rep_lds = reinterpret_cast<uint32_t*>(smem);
  const uint32_t rep_bytes = ((uint32_t)a.nreps * 4u + 15u) & ~15u;
  unsigned char* buf0 = smem + rep_bytes;
  const uint32_t bb = (uint32_t)a.lds_tile_bytes;
  const int64_t x = blockIdx.x & 7u;
  const int64_t nj = gridDim.x >> 3;
  auto item_at = [&](int64_t k) -> int64_t {
    int64_t it;
    if (a.xcd_per > 0) {
      int64_t L = (int64_t)(blockIdx.x >> 3) + k * nj;
      if (L >= a.xcd_per) return -1;
      it = x * a.xcd_per + L;
    } else {
      it = (int64_t)blockIdx.x + k * (int64_t)gridDim.x;
    }
    if (it >= a.nitems) return -1;
    return a.reverse ? a.nitems - 1 - it : it;
  };
  int64_t it = item_at(0);
  if (it < 0) return;
  for (int i = threadIdx.x; i < a.nreps; i += blockDim.x) rep_lds[i] = a.reps[i];
  const bool whole = (g.bl == g.n);
  const cptr<T> coef = as_const(a.coef);
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, it, &cube0, &orbit, &ncub);
  cptr<GroupDev> od = as_const(a.orbits + orbit);
  int ntl = whole ? ncub : od->ntiles;
  bool ragged = od->ragged != 0;
  issue_item_lds<T, D>(g, od, whole, ntl, ragged, a.in + cube0 * g.cube_elems, buf0);
  uint32_t par = 0;
  for (int64_t k = 0;; ++k) {
    clear_terms_flag(a.sparse);
    const int64_t nx = item_at(k + 1);
    int64_t cube0n = 0;
    int orbitn = 0, ncubn = 0, ntln = 0;
    cptr<GroupDev> odn = od;
    bool raggedn = false;
    int pending = 0;
    if (nx >= 0) {
      decode_item(g, nx, &cube0n, &orbitn, &ncubn);
      odn = as_const(a.orbits + orbitn);
      ntln = whole ? ncubn : odn->ntiles;
      raggedn = odn->ragged != 0;
      pending = issue_item_lds<T, D>(g, odn, whole, ntln, raggedn, a.in + cube0n * g.cube_elems,
                                     buf0 + (par ^ 1u) * bb);
    }
    // everything but the next item's loads has completed: this item's tiles
    // are in LDS (and the previous item's stores have left)
    wait_vmcnt_atmost(pending);
    lds_barrier();
    T* lds = reinterpret_cast<T*>(buf0 + par * bb);
    const bool bad = combine_item<T, D, CHAIN, false>(g, od, rep_lds, coef, a.nstages, ncub, lds);
    if (a.sparse != 0u && item_needs_terms(a.sparse, bad)) {  // (drains the prefetch: rare path)
      redo_item<T, D, CHAIN, false>(g, od, rep_lds, coef, a.nstages, ncub,
                                    a.in + cube0 * g.cube_elems, lds);
    }
    lds_barrier();
    store_item_lds<T, D, NTS>(g, od, whole, ntl, ragged, a.out + cube0 * g.cube_elems, lds);
    // the buffer is refilled two items on: every wave has read it by then
    lds_barrier();
    if (nx < 0) break;
    cube0 = cube0n;
    ncub = ncubn;
    od = odn;
    ntl = ntln;
    ragged = raggedn;
    par ^= 1u;
  }
}

// Persistent, software-pipelined: the loads of the next item are in flight
// while the current item is combined and stored.  gridDim.x is a multiple of
// 8.  Per item:
//   A. stage the next item's tile table and this item's representatives in
//      LDS, wait for this item's tiles and write them to LDS;   barrier
//   B. issue the loads of the next item (registers, no wait)
//   C. combine this item in LDS (LDS and scalar loads only); barrier
//   D. store this item;                                       barrier
// LDS: [tiles | representatives (g.rep_lds entries)].
template <typename T, int D, int VW, bool CHAIN, int MAXC>
__global__ void __launch_bounds__(kThreads) k_pipe(const ExecArgs<T> a) {
  typedef typename VecT<T, VW>::type V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int32_t tinfo[2][2 * kMaxDF];
  T* lds = reinterpret_cast<T*>(smem);
  uint32_t* rep_lds = reinterpret_cast<uint32_t*>(smem + (size_t)a.lds_tile_bytes);
  const Geom& g = a.g;
  const int64_t x = blockIdx.x & 7u;
  const int64_t nj = gridDim.x >> 3;
  auto item_at = [&](int64_t k) -> int64_t {
    int64_t it;
    if (a.xcd_per > 0) {
      int64_t L = (int64_t)(blockIdx.x >> 3) + k * nj;
      if (L >= a.xcd_per) return -1;
      it = x * a.xcd_per + L;
    } else {
      it = (int64_t)blockIdx.x + k * (int64_t)gridDim.x;
    }
    if (it >= a.nitems) return -1;
    return a.reverse ? a.nitems - 1 - it : it;
  };
  const cptr<T> coef = as_const(a.coef);
  int64_t k = 0;
  int64_t it = item_at(0);
  if (it < 0) return;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, it, &cube0, &orbit, &ncub);
  const GroupDev* od = a.orbits + orbit;
  stage_tinfo(tinfo[0], od);
  __syncthreads();
  V buf[MAXC];
  int lo[MAXC];
  int ntiles = as_const(od)->ntiles;
  bool ragged = as_const(od)->ragged != 0;
  uint32_t nchunks = (uint32_t)ncub * (uint32_t)ntiles * (uint32_t)g.rows * (uint32_t)g.vpr;
  issue_loads<T, D, VW, MAXC>(g, tinfo[0], ntiles, ragged, nchunks, a.in + cube0 * g.cube_elems,
                              buf, lo);
  int par = 0;
  while (true) {
    clear_terms_flag(a.sparse);
    const int64_t nx = item_at(k + 1);
    int64_t cube0n = 0;
    int orbitn = 0, ncubn = 0;
    const GroupDev* odn = od;
    // A.
    if (nx >= 0) {
      decode_item(g, nx, &cube0n, &orbitn, &ncubn);
      odn = a.orbits + orbitn;
      stage_tinfo(tinfo[par ^ 1], odn);
    }
    {
      cptr<GroupDev> cod = as_const(od);
      const int norb = cod->norb;
      for (int kk = 0; kk < norb; ++kk) {
        const int rc = cod->rep_cnt[kk];
        const uint32_t* rsrc = a.reps + cod->rep_off[kk];
        uint32_t* rdst = rep_lds + cod->rep_base[kk];
        for (int i = threadIdx.x; i < rc; i += kThreads) rdst[i] = rsrc[i];
      }
    }
    fill_lds<T, VW, MAXC>(buf, lo, lds);
    // Every load of the previous phase has landed.  Saying so explicitly
    // (s_waitcnt vmcnt(0), gfx9 encoding) keeps the compiler from waiting
    // between the prefetch loads below, which reuse the same registers.
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    // B.
    int ntilesn = 0;
    bool raggedn = false;
    uint32_t nchunksn = 0;
    if (nx >= 0) {
      ntilesn = as_const(odn)->ntiles;
      raggedn = as_const(odn)->ragged != 0;
      nchunksn = (uint32_t)ncubn * (uint32_t)ntilesn * (uint32_t)g.rows * (uint32_t)g.vpr;
      issue_loads<T, D, VW, MAXC>(g, tinfo[par ^ 1], ntilesn, raggedn, nchunksn,
                                  a.in + cube0n * g.cube_elems, buf, lo);
    }
    // C.
    const bool bad =
        combine_item<T, D, CHAIN, true>(g, as_const(od), rep_lds, coef, a.nstages, ncub, lds);
    if (item_needs_terms(a.sparse, bad)) {
      redo_item<T, D, CHAIN, true>(g, as_const(od), rep_lds, coef, a.nstages, ncub,
                                   a.in + cube0 * g.cube_elems, lds);
      __syncthreads();
    }
    // D.
    store_item<T, D, VW, true>(g, tinfo[par], ntiles, ragged, nchunks,
                               a.out + cube0 * g.cube_elems, lds);
    __syncthreads();
    if (nx < 0) break;
    ++k;
    cube0 = cube0n;
    ncub = ncubn;
    od = odn;
    ntiles = ntilesn;
    ragged = raggedn;
    nchunks = nchunksn;
    par ^= 1;
  }
}

// Batched: one work item of the cost-sorted list.  Whole-cube items (every
// block whose cube fits) are copied as one contiguous run straight into LDS,
// with their representative lists behind them; tile-orbit items of larger
// cubes go through registers.
template <typename T, int D, int VW>
__device__ __forceinline__ void batched_item(const BatchArgs<T>& a, int64_t it,
                                             unsigned char* smem) {
  typedef typename VecT<T, VW>::type V;
  T* lds = reinterpret_cast<T*>(smem);
  const cptr<BatchItem> item = as_const(a.items) + it;
  const int blk = item->block;
  const int64_t icube0 = item->cube0;
  const int incubes = item->ncubes;
  const Geom g = load_geom(as_const(a.blocks)[blk].g);
  const T* src = as_const(a.in)[blk] + icube0 * g.cube_elems;
  T* dst = as_const(a.out)[blk] + icube0 * g.cube_elems;
  const GroupDev* od = a.orbits + item->group;
  cptr<GroupDev> cod = as_const(od);
  const cptr<T> coef = as_const(a.coef);
  unsigned char* rep_lds = smem + a.lds_tile_bytes;
  clear_terms_flag(a.sparse);
  if (g.bl == g.n) {
    const uint32_t span = (uint32_t)incubes * (uint32_t)g.cube_elems;
    set_memory_priority();
    const int shift = flat_issue<T, true>(src, span, smem);  // one run: whole lines
    issue_reps_lds(cod, a.reps, rep_lds);
    set_compute_priority();
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): everything is in LDS
    __syncthreads();
    const bool bad = combine_item<T, D, false, true>(
        g, cod, reinterpret_cast<const uint32_t*>(rep_lds), coef, 1, incubes, lds + shift);
    if (item_needs_terms(a.sparse, bad)) {
      redo_item<T, D, false, true>(g, cod, reinterpret_cast<const uint32_t*>(rep_lds), coef, 1,
                                   incubes, src, lds + shift);
      __syncthreads();
    }
    set_memory_priority();
    flat_store<T, true>(dst, span, smem, shift);
    set_compute_priority();
    return;
  }
  int32_t* tinfo = reinterpret_cast<int32_t*>(rep_lds);  // tile table (no lists needed)
  stage_tinfo(tinfo, od);
  __syncthreads();
  const int ntiles = cod->ntiles;
  const bool ragged = cod->ragged != 0;
  const uint32_t nchunks =
      (uint32_t)incubes * (uint32_t)ntiles * (uint32_t)g.rows * (uint32_t)g.vpr;
  for (uint32_t c0 = 0; c0 < nchunks; c0 += kUnroll * kThreads) {
    V buf[kUnroll];
    int lo[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint32_t c = c0 + threadIdx.x + u * kThreads;
      int go = 0;
      int l = 0;
      bool ok = (c < nchunks) && chunk_addr<D, VW>(g, c, ntiles, tinfo, tinfo + kMaxDF, ragged, &go, &l);
      lo[u] = ok ? l : -1;
      if (ok) buf[u] = *reinterpret_cast<const V*>(src + go);
    }
    fill_lds<T, VW, kUnroll>(buf, lo, lds);
  }
  __syncthreads();
  const bool bad = combine_item<T, D, false, false>(g, cod, a.reps, coef, 1, incubes, lds);
  if (item_needs_terms(a.sparse, bad)) {
    redo_item<T, D, false, false>(g, cod, a.reps, coef, 1, incubes, src, lds);
    __syncthreads();
  }
  store_item<T, D, VW, true>(g, tinfo, ntiles, ragged, nchunks, dst, lds);
}

// One item per workgroup (the hardware dispatcher is the queue), or, with
// PERSIST, a grid sized to the occupancy whose workgroups walk the list:
// workgroup j of XCD x takes items j, j + stride, ... of that XCD's
// contiguous range (stride = workgroups per XCD), so the workgroups of one
// XCD work on neighbouring items at any time.
template <typename T, int D, int VW, bool PERSIST>
__global__ void __launch_bounds__(kThreads) k_batched(const BatchArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if constexpr (!PERSIST) {
    int64_t it;
    if (a.xcd_per > 0)
      it = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
    else
      it = blockIdx.x;
    if (it >= a.nitems) return;
    batched_item<T, D, VW>(a, it, smem);
  } else {
    int64_t first, stride, end;
    if (a.xcd_per > 0) {
      const int64_t x = blockIdx.x & 7u;
      first = x * a.xcd_per + (blockIdx.x >> 3);
      stride = gridDim.x >> 3;
      end = (x + 1) * a.xcd_per < a.nitems ? (x + 1) * a.xcd_per : a.nitems;
    } else {
      first = blockIdx.x;
      stride = gridDim.x;
      end = a.nitems;
    }
    for (int64_t it = first; it < end; it += stride) {
      batched_item<T, D, VW>(a, it, smem);
      __syncthreads();  // the next item's loads reuse the LDS
    }
  }
}

// Coefficient gradient: c_p = <gr, P_p x> for every permutation p of the
// group -- the derivative of <gr, S(x)> with respect to the coefficient of p.
// Over one element orbit, with v_sigma = x[sigma . r] and u_tau =
// gr[tau . r], the terms are sum_tau u_tau v_(tau o p); every element of the
// orbit appears |H| times among the tau (H: the permutations that fix r),
// so the orbit's share is that sum / |H|.
template <int D, int P, int... TAU>
__device__ __forceinline__ double cgrad_row(const double* u, const double* v,
                                           std::integer_sequence<int, TAU...>) {
  double s = 0.0;
  ((s = fma_t(u[TAU], v[Compose<D, TAU, P>::value], s)), ...);
  return s;
}

template <int D, int... P>
__device__ __forceinline__ void cgrad_rows(double* acc, const double* u, const double* v, double w,
                                           std::integer_sequence<int, P...>) {
  ((acc[P] = fma_t(w, cgrad_row<D, P>(u, v, std::make_integer_sequence<int, Fact<D>::v>{}), acc[P])),
   ...);
}

template <typename T, int D>
__global__ void __launch_bounds__(kThreads) k_cgrad(const CGradArgs<T> a) {
  constexpr int DF = Fact<D>::v;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  const Geom& g = a.g;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, item, &cube0, &orbit, &ncub);
  const cptr<GroupDev> od = as_const(a.orbits + orbit);
  const bool whole = (g.bl == g.n);
  const int ntl = whole ? ncub : od->ntiles;
  const bool ragged = od->ragged != 0;
  unsigned char* ldsx = smem;
  unsigned char* ldsg = smem + a.lds_tile_bytes;
  unsigned char* rep_lds = smem + 2 * a.lds_tile_bytes;
  const uint32_t span = (uint32_t)ncub * (uint32_t)g.cube_elems;
  int sx = 0, sg = 0;
  set_memory_priority();
  if (whole) {
    sx = flat_issue<T>(a.x + cube0 * g.cube_elems, span, ldsx);
    sg = flat_issue<T>(a.gr + cube0 * g.cube_elems, span, ldsg);
  } else {
    issue_item_lds<T, D>(g, od, false, ntl, ragged, a.x + cube0 * g.cube_elems, ldsx);
    issue_item_lds<T, D>(g, od, false, ntl, ragged, a.gr + cube0 * g.cube_elems, ldsg);
  }
  issue_reps_lds(od, a.reps, rep_lds);
  set_compute_priority();
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): everything is in LDS
  __syncthreads();
  const T* X = reinterpret_cast<const T*>(ldsx) + sx;
  const T* U = reinterpret_cast<const T*>(ldsg) + sg;
  const uint32_t* reps = reinterpret_cast<const uint32_t*>(rep_lds);
  double acc[DF];
#pragma unroll
  for (int p = 0; p < DF; ++p) acc[p] = 0.0;
  const int norb = od->norb;
  for (int k = 0; k < norb; ++k) {
    int32_t sb[DF];
#pragma unroll
    for (int r = 0; r < DF; ++r) sb[r] = od->slot_base[k][r];
    const uint32_t rep_cnt = (uint32_t)od->rep_cnt[k];
    const uint32_t nrep = (uint32_t)ncub * rep_cnt * (uint32_t)g.inner;
    const FastDiv fdr = load_fd(od->fd_rep[k]);
    const uint32_t* rp = reps + od->rep_base[k];
    const int eq = od->eqmask[k];
    for (uint32_t i = threadIdx.x; i < nrep; i += blockDim.x) {
      uint32_t ci, ri, si;
      split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
      uint32_t pk = rp[ri];
      int l[D];
#pragma unroll
      for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
      int addr[DF];
      orbit_addrs<D>(g, (int)ci * g.cube_lds + (int)si, sb, l, addr,
                     std::make_integer_sequence<int, DF>{});
      double v[DF], u[DF];
#pragma unroll
      for (int r = 0; r < DF; ++r) {
        v[r] = (double)X[addr[r]];
        u[r] = (double)U[addr[r]];
      }
      // |H|: equal global coordinates are neighbours in a representative
      // (equal blocks, local coordinates non-decreasing within them)
      int h = 1, run = 1;
#pragma unroll
      for (int m = 1; m < D; ++m) {
        if (((eq >> (m - 1)) & 1) && l[m] == l[m - 1]) {
          ++run;
          h *= run;
        } else {
          run = 1;
        }
      }
      cgrad_rows<D>(acc, u, v, 1.0 / (double)h, std::make_integer_sequence<int, DF>{});
    }
  }
  // workgroup sum: within each wave, then across the waves through LDS
  __syncthreads();  // every wave is done with the tiles
  double* red = reinterpret_cast<double*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < DF; ++p) {
    double s = acc[p];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave * DF + p] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < DF) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w * DF + threadIdx.x];
    // one of kGradSlots partial sums per permutation: spreads the atomic
    // adds of the workgroups over many addresses
    unsafeAtomicAdd(a.grad + (blockIdx.x & (kGradSlots - 1)) * DF + threadIdx.x, s);
  }
}

// Coefficient gradient with one tile buffer, for tiled items of one tile
// orbit whose chunks take one pass of the workgroup (every thread holds at
// most one chunk per tile) and whose element orbits are at most two per
// thread.  The tiles of x go straight into LDS while those of the upstream
// gradient go into registers, all loads in flight together; every thread
// gathers the d! values of x of its element orbits into registers, the
// gradient's tiles then take x's place in LDS, and each element orbit's
// terms are formed as in k_cgrad.  Half of k_cgrad's LDS, so twice its
// workgroups fit a CU (the plan's own tiling: no packed items needed).
// LDS: [tiles (lds_tile_bytes) | representative list]; the partial sums of
// the waves reuse it at the end.  At least six waves per SIMD (the second
// launch bound): unbounded, the compiler takes 184 VGPRs (two waves) for
// what fits in 78 without spilling, and the LDS would allow six
// workgroups per CU.
static_assert(kCgSplitThreads == kThreads, "k_cgrad_split runs kThreads per workgroup");

template <typename T, int D>
__global__ void __launch_bounds__(kThreads, 6) k_cgrad_split(const CGradArgs<T> a) {
  constexpr int DF = Fact<D>::v;
  constexpr int VW = 16 / sizeof(T);
  typedef typename VecT<T, VW>::type V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  const Geom& g = a.g;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, item, &cube0, &orbit, &ncub);
  const cptr<GroupDev> od = as_const(a.orbits + orbit);
  const int ntl = od->ntiles;
  const bool ragged = od->ragged != 0;
  T* lds = reinterpret_cast<T*>(smem);
  unsigned char* rep_lds = smem + a.lds_tile_bytes;
  // 1. x's tiles to LDS, the gradient's chunks to registers (chunk tid of
  //    every tile: the plan allows this kernel only where rows * vpr fits
  //    the workgroup), the representative list to LDS
  int l[D];
  chunk_coords<D, VW>(g, threadIdx.x, l);
  const int off = chunk_offset<D>(g, l);
  const bool cin = threadIdx.x < (uint32_t)g.rows * (uint32_t)g.vpr;
  set_memory_priority();
  issue_item_lds<T, D, false>(g, od, false, ntl, ragged, a.x + cube0 * g.cube_elems, smem);
  const T* gsrc = a.gr + cube0 * g.cube_elems;
  V gb[kCgSplitTiles];
#pragma unroll
  for (int t = 0; t < kCgSplitTiles; ++t) {
    if (t < ntl && cin && (!ragged || chunk_inside<D>(l, od->tile_ext[t], g.inner)))
      gb[t] = *reinterpret_cast<const V*>(gsrc + od->tile_off[t] + off);
  }
  issue_reps_lds(od, a.reps, rep_lds);
  set_compute_priority();
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): x and the lists in LDS, gb loaded
  __syncthreads();
  // 2. the x values of this thread's element orbits
  int32_t sb[DF];
#pragma unroll
  for (int r = 0; r < DF; ++r) sb[r] = od->slot_base[0][r];
  const uint32_t rep_cnt = (uint32_t)od->rep_cnt[0];
  const uint32_t* rp = reinterpret_cast<const uint32_t*>(rep_lds);
  const int eq = od->eqmask[0];
  double v[kCgSplitUnits][DF];
  int addr[kCgSplitUnits][DF];
  double w[kCgSplitUnits];
#pragma unroll
  for (int u = 0; u < kCgSplitUnits; ++u) {
    const uint32_t i = threadIdx.x + u * blockDim.x;
    w[u] = 0.0;
    if (i < rep_cnt) {
      const uint32_t pk = rp[i];
      int lr[D];
#pragma unroll
      for (int m = 0; m < D; ++m) lr[m] = (int)((pk >> (8 * m)) & 255u);
      orbit_addrs<D>(g, 0, sb, lr, addr[u], std::make_integer_sequence<int, DF>{});
#pragma unroll
      for (int r = 0; r < DF; ++r) v[u][r] = (double)lds[addr[u][r]];
      // |H| as in k_cgrad
      int h = 1, run = 1;
#pragma unroll
      for (int m = 1; m < D; ++m) {
        if (((eq >> (m - 1)) & 1) && lr[m] == lr[m - 1]) {
          ++run;
          h *= run;
        } else {
          run = 1;
        }
      }
      w[u] = 1.0 / (double)h;
    }
  }
  __syncthreads();  // every wave is done with x
  // 3. the gradient's tiles take x's place
#pragma unroll
  for (int t = 0; t < kCgSplitTiles; ++t) {
    if (t < ntl && cin && (!ragged || chunk_inside<D>(l, od->tile_ext[t], g.inner)))
      *reinterpret_cast<V*>(lds + t * g.ts + (int)threadIdx.x * VW) = gb[t];
  }
  __syncthreads();
  double acc[DF];
#pragma unroll
  for (int p = 0; p < DF; ++p) acc[p] = 0.0;
#pragma unroll
  for (int u = 0; u < kCgSplitUnits; ++u) {
    if (w[u] != 0.0) {
      double gu[DF];
#pragma unroll
      for (int r = 0; r < DF; ++r) gu[r] = (double)lds[addr[u][r]];
      cgrad_rows<D>(acc, gu, v[u], w[u], std::make_integer_sequence<int, DF>{});
    }
  }
  // 4. workgroup sum, as in k_cgrad
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < DF; ++p) {
    double s = acc[p];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[wave * DF + p] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < DF) {
    double s = 0.0;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) s += red[wv * DF + threadIdx.x];
    unsafeAtomicAdd(a.grad + (blockIdx.x & (kGradSlots - 1)) * DF + threadIdx.x, s);
  }
}

// Zero n doubles (grid-stride).
__global__ void __launch_bounds__(kThreads) k_zero_f64(double* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

// grad[p] = sum over the kGradSlots partial sums of p (workgroup p).
__global__ void __launch_bounds__(kThreads) k_grad_reduce(const double* part, double* grad, int df) {
  __shared__ double red[kThreads];
  const int p = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < kGradSlots; i += kThreads) s += part[i * df + p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[p] = red[0];
}

// Lexicographic rank of a strictly increasing tuple X of [0, N) among all
// C(N, d) of them: the tuples after X, read backwards as N-1-X, are counted
// in the combinatorial number system (sum over m of C(y_m, m+1) for the
// increasing y), so rank = C(N, d) - 1 - that count.  Exact in 64 bits
// for N < 2^16.
__device__ __forceinline__ uint64_t binom_upto4(uint64_t y, int k) {
  if (k == 1) return y;
  if (k == 2) return y * (y - 1) / 2;
  if (k == 3) return y < 3 ? 0 : y * (y - 1) / 2 * (y - 2) / 3;
  return y < 4 ? 0 : y * (y - 1) / 2 * (y - 2) / 3 * (y - 3) / 4;
}

template <int D>
__device__ __forceinline__ int64_t increasing_rank(const int (&X)[D], int n, int64_t ncomb) {
  uint64_t c = 0;
#pragma unroll
  for (int m = 0; m < D; ++m) c += binom_upto4((uint64_t)(n - 1 - X[D - 1 - m]), m + 1);
  return ncomb - 1 - (int64_t)c;
}

// Origin (group coordinates) of the identity tile of orbit k of an item.
template <int D>
__device__ __forceinline__ void orbit_origin(const Geom& g, cptr<GroupDev> gd, int k,
                                             int (&org)[D]) {
  const uint32_t off = (uint32_t)gd->tile_off[(uint32_t)gd->slot_base[k][0] / (uint32_t)g.ts];
#pragma unroll
  for (int m = 0; m < D; ++m) org[m] = (int)((off / (uint32_t)g.gst[m]) % (uint32_t)g.n);
}

template <typename T, int D, int... TAU>
__device__ __forceinline__ void unpack_rows(const T (&a)[Fact<D>::v], T v, T* lds,
                                            const int (&addr)[Fact<D>::v],
                                            std::integer_sequence<int, TAU...>) {
  // w_tau = a(tau^-1) v: the one input of the element orbit is the packed
  // value at its increasing tuple (the identity's slot); a zero coefficient
  // is not a term, so it gives 0 even for a non-finite v
  ((lds[addr[TAU]] = (a[GinvMul<D, TAU, 0>::value] != T(0)) ? a[GinvMul<D, TAU, 0>::value] * v
                                                             : T(0)),
   ...);
}

template <typename T, int D, int... S>
__device__ __forceinline__ T pack_row(const T (&a)[Fact<D>::v], const T (&v)[Fact<D>::v],
                                      std::integer_sequence<int, S...>) {
  // (S^T f)[x] = sum_sigma a(sigma^-1) f[sigma . x], over the terms only
  T acc = T(0);
  ((acc = (a[GinvMul<D, S, 0>::value] != T(0)) ? fma_t(a[GinvMul<D, S, 0>::value], v[S], acc) : acc),
   ...);
  return acc;
}

// Unpacking: full = S(E(packed)), E placing the packed values at the
// strictly increasing group positions of a zero tensor.  An element orbit
// {sigma . x} (x sorted) holds one packed value when x is strictly
// increasing and none otherwise, so its outputs are a(tau^-1) v or zero.
// Work items, LDS layout and stores as in k_lds; nothing is read from the
// full tensor.  One work item per workgroup, XCD-grouped.
template <typename T, int D, bool NTS>
__global__ void __launch_bounds__(kMaxThreads) k_unpack(const PackArgs<T> a) {
  constexpr int DF = Fact<D>::v;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  const Geom& g = a.g;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, item, &cube0, &orbit, &ncub);
  const cptr<GroupDev> od = as_const(a.orbits + orbit);
  const bool whole = (g.bl == g.n);
  const int ntl = whole ? ncub : od->ntiles;
  const bool ragged = od->ragged != 0;
  T* dst = a.full_out + cube0 * g.cube_elems;
  // whole cubes are laid out as the contiguous store expects them
  const int shift = whole ? flat_shift<T>(dst) : 0;
  T* lds = reinterpret_cast<T*>(smem) + shift;
  unsigned char* rep_lds = smem + a.lds_tile_bytes;
  issue_reps_lds(od, a.reps, rep_lds);
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  T co[DF];
  const cptr<T> coef = as_const(a.coef);
#pragma unroll
  for (int r = 0; r < DF; ++r) co[r] = coef[r];
  const uint32_t* reps = reinterpret_cast<const uint32_t*>(rep_lds);
  const int norb = od->norb;
  for (int k = 0; k < norb; ++k) {
    int32_t sb[DF];
#pragma unroll
    for (int r = 0; r < DF; ++r) sb[r] = od->slot_base[k][r];
    int org[D];
    orbit_origin<D>(g, od, k, org);
    const uint32_t rep_cnt = (uint32_t)od->rep_cnt[k];
    const FastDiv fdr = load_fd(od->fd_rep[k]);
    const uint32_t* rp = reps + od->rep_base[k];
    const uint32_t nrep = (uint32_t)ncub * rep_cnt * (uint32_t)g.inner;
    // kUnpackBatch units per thread at a time: their packed values are all
    // requested before the first is used, so the gathers overlap
    for (uint32_t i0 = 0; i0 < nrep; i0 += kUnpackBatch * blockDim.x) {
      T v[kUnpackBatch];
      bool strict[kUnpackBatch];
#pragma unroll
      for (int u = 0; u < kUnpackBatch; ++u) {
        const uint32_t i = i0 + threadIdx.x + u * blockDim.x;
        v[u] = T(0);
        strict[u] = false;
        if (i < nrep) {
          uint32_t ci, ri, si;
          split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
          const uint32_t pk = rp[ri];
          int X[D];
#pragma unroll
          for (int m = 0; m < D; ++m) X[m] = org[m] + (int)((pk >> (8 * m)) & 255u);
          bool st = true;
#pragma unroll
          for (int m = 0; m + 1 < D; ++m) st = st && (X[m] < X[m + 1]);
          strict[u] = st;
          if (st) {
            const int64_t r = increasing_rank<D>(X, g.n, a.ncomb);
            v[u] = a.packed_in[((cube0 + (int64_t)ci) * a.ncomb + r) * g.inner + (int64_t)si];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kUnpackBatch; ++u) {
        const uint32_t i = i0 + threadIdx.x + u * blockDim.x;
        if (i < nrep) {
          uint32_t ci, ri, si;
          split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
          const uint32_t pk = rp[ri];
          int l[D];
#pragma unroll
          for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
          int addr[DF];
          orbit_addrs<D>(g, (int)ci * g.cube_lds + (int)si, sb, l, addr,
                         std::make_integer_sequence<int, DF>{});
          if (strict[u]) {
            unpack_rows<T, D>(co, v[u], lds, addr, std::make_integer_sequence<int, DF>{});
          } else {
#pragma unroll
            for (int r = 0; r < DF; ++r) lds[addr[r]] = T(0);
          }
        }
      }
    }
  }
  __syncthreads();
  set_memory_priority();
  if (whole)
    flat_store<T, NTS>(dst, (uint32_t)ncub * (uint32_t)g.cube_elems, smem, shift);
  else
    store_item_lds<T, D, NTS>(g, od, whole, ntl, ragged, dst, lds);
}

// Unpacking, persistent: each workgroup takes one item template (a tile
// orbit, or the whole cube) and walks its XCD's range of cubes.  The
// template's element orbits (representative, inner index) are the same in
// every cube, so each thread works out once which packed entry each of its
// units reads (its rank) and whether the unit is strictly increasing; the
// packed values of the next cube are requested before the current item's
// stores, so that their trip to memory overlaps the stores instead of
// following them.  Templates get workgroups in proportion to their tiles
// (tmpl_wg: prefix sums, multiples of 8).  Output as in k_unpack.
template <typename T, int D, bool NTS>
__global__ void __launch_bounds__(kMaxThreads) k_unpack_persist(const PackArgs<T> a) {
  constexpr int DF = Fact<D>::v;
  constexpr int U = kUnpackCubeUnits;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const Geom& g = a.g;
  int t = 0;
  while (t + 1 < a.ntmpl && (int)blockIdx.x >= a.tmpl_wg[t + 1]) ++t;
  const uint32_t w = blockIdx.x - (uint32_t)a.tmpl_wg[t];
  const int64_t nloc = (int64_t)((a.tmpl_wg[t + 1] - a.tmpl_wg[t]) >> 3);
  const int64_t per = a.xcd_per;
  int64_t c = (int64_t)(w & 7u) * per + (int64_t)(w >> 3);
  int64_t cend = (int64_t)(w & 7u) * per + per;
  if (cend > g.ncubes) cend = g.ncubes;
  if (c >= cend) return;
  const cptr<GroupDev> od = as_const(a.orbits + t);
  const bool whole = (g.bl == g.n);
  const bool ragged = od->ragged != 0;
  const int ntl = whole ? 1 : od->ntiles;
  const uint32_t rep_cnt = (uint32_t)od->rep_cnt[0];
  const uint32_t nunit = rep_cnt * (uint32_t)g.inner;
  const FastDiv fdr = load_fd(od->fd_rep[0]);
  const uint32_t* rp = a.reps + od->rep_off[0];
  int32_t sb[DF];
#pragma unroll
  for (int r = 0; r < DF; ++r) sb[r] = od->slot_base[0][r];
  int org[D];
  orbit_origin<D>(g, od, 0, org);
  T co[DF];
  const cptr<T> coef = as_const(a.coef);
#pragma unroll
  for (int r = 0; r < DF; ++r) co[r] = coef[r];
  // per unit: its representative (local coordinates, one byte per axis),
  // its offset in a cube's packed values, or -1 where the tuple repeats an
  // index (the orbit's outputs are zero) or -2 where the unit does not exist
  uint32_t pk[U];
  int32_t poff[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t i = threadIdx.x + (uint32_t)u * blockDim.x;
    pk[u] = 0;
    poff[u] = -2;
    if (i < nunit) {
      uint32_t ci, ri, si;
      split_unit(g, i, rep_cnt, fdr, 1, &ci, &ri, &si);
      pk[u] = rp[ri];
      int X[D];
#pragma unroll
      for (int m = 0; m < D; ++m) X[m] = org[m] + (int)((pk[u] >> (8 * m)) & 255u);
      bool st = true;
#pragma unroll
      for (int m = 0; m + 1 < D; ++m) st = st && (X[m] < X[m + 1]);
      poff[u] = st ? (int32_t)(increasing_rank<D>(X, g.n, a.ncomb) * g.inner + (int64_t)si) : -1;
    }
  }
  const int64_t pstride = a.ncomb * (int64_t)g.inner;
  T v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = poff[u] >= 0 ? a.packed_in[c * pstride + poff[u]] : T(0);
  for (;;) {
    T* dst = a.full_out + c * g.cube_elems;
    const int shift = whole ? flat_shift<T>(dst) : 0;
    T* lds = reinterpret_cast<T*>(smem) + shift;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (poff[u] == -2) continue;
      const uint32_t i = threadIdx.x + (uint32_t)u * blockDim.x;
      const uint32_t si = (g.inner != 1) ? i - fdiv(i, g.fd_inner) * (uint32_t)g.inner : 0u;
      int l[D];
#pragma unroll
      for (int m = 0; m < D; ++m) l[m] = (int)((pk[u] >> (8 * m)) & 255u);
      int addr[DF];
      orbit_addrs<D>(g, (int)si, sb, l, addr, std::make_integer_sequence<int, DF>{});
      if (poff[u] >= 0) {
        unpack_rows<T, D>(co, v[u], lds, addr, std::make_integer_sequence<int, DF>{});
      } else {
#pragma unroll
        for (int r = 0; r < DF; ++r) lds[addr[r]] = T(0);
      }
    }
    __syncthreads();
    const int64_t cn = c + nloc;
    if (cn < cend) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = poff[u] >= 0 ? a.packed_in[cn * pstride + poff[u]] : T(0);
    }
    if (whole)
      flat_store<T, NTS>(dst, (uint32_t)g.cube_elems, smem, shift);
    else
      store_item_lds<T, D, NTS>(g, od, false, ntl, ragged, dst, lds);
    if (cn >= cend) break;
    // every thread has read its part of this item from LDS
    __syncthreads();
    c = cn;
  }
}

// Packing, the adjoint of unpacking: packed = E^T S^T full -- for every
// strictly increasing x, sum_sigma a(sigma^-1) full[sigma . x].  The item's
// tiles are loaded as in k_lds; nothing is stored to the full tensor.
template <typename T, int D>
__global__ void __launch_bounds__(kMaxThreads) k_pack(const PackArgs<T> a) {
  constexpr int DF = Fact<D>::v;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int64_t item;
  if (a.xcd_per > 0)
    item = (int64_t)(blockIdx.x & 7u) * a.xcd_per + (int64_t)(blockIdx.x >> 3);
  else
    item = blockIdx.x;
  if (item >= a.nitems) return;
  const Geom& g = a.g;
  int64_t cube0;
  int orbit, ncub;
  decode_item(g, item, &cube0, &orbit, &ncub);
  const cptr<GroupDev> od = as_const(a.orbits + orbit);
  const bool whole = (g.bl == g.n);
  const int ntl = whole ? ncub : od->ntiles;
  const bool ragged = od->ragged != 0;
  unsigned char* rep_lds = smem + a.lds_tile_bytes;
  const uint32_t span = (uint32_t)ncub * (uint32_t)g.cube_elems;
  int shift = 0;
  set_memory_priority();
  if (whole)
    shift = flat_issue<T>(a.full_in + cube0 * g.cube_elems, span, smem);
  else
    issue_item_lds<T, D>(g, od, whole, ntl, ragged, a.full_in + cube0 * g.cube_elems, smem);
  issue_reps_lds(od, a.reps, rep_lds);
  set_compute_priority();
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  const T* lds = reinterpret_cast<const T*>(smem) + shift;
  T co[DF];
  const cptr<T> coef = as_const(a.coef);
#pragma unroll
  for (int r = 0; r < DF; ++r) co[r] = coef[r];
  const uint32_t* reps = reinterpret_cast<const uint32_t*>(rep_lds);
  const int norb = od->norb;
  for (int k = 0; k < norb; ++k) {
    int32_t sb[DF];
#pragma unroll
    for (int r = 0; r < DF; ++r) sb[r] = od->slot_base[k][r];
    int org[D];
    orbit_origin<D>(g, od, k, org);
    const uint32_t rep_cnt = (uint32_t)od->rep_cnt[k];
    const FastDiv fdr = load_fd(od->fd_rep[k]);
    const uint32_t* rp = reps + od->rep_base[k];
    const uint32_t nrep = (uint32_t)ncub * rep_cnt * (uint32_t)g.inner;
    for (uint32_t i = threadIdx.x; i < nrep; i += blockDim.x) {
      uint32_t ci, ri, si;
      split_unit(g, i, rep_cnt, fdr, ncub, &ci, &ri, &si);
      const uint32_t pk = rp[ri];
      int l[D], X[D];
#pragma unroll
      for (int m = 0; m < D; ++m) {
        l[m] = (int)((pk >> (8 * m)) & 255u);
        X[m] = org[m] + l[m];
      }
      bool strict = true;
#pragma unroll
      for (int m = 0; m + 1 < D; ++m) strict = strict && (X[m] < X[m + 1]);
      if (!strict) continue;
      int addr[DF];
      T v[DF];
      orbit_addrs<D>(g, (int)ci * g.cube_lds + (int)si, sb, l, addr,
                     std::make_integer_sequence<int, DF>{});
#pragma unroll
      for (int r = 0; r < DF; ++r) v[r] = lds[addr[r]];
      const int64_t rk = increasing_rank<D>(X, g.n, a.ncomb);
      a.packed_out[((cube0 + (int64_t)ci) * a.ncomb + rk) * g.inner + (int64_t)si] =
          pack_row<T, D>(co, v, std::make_integer_sequence<int, DF>{});
    }
  }
}

// ------------------------------------------------------------ dispatch
template <typename T, int D, bool CHAIN, bool NTS>
const void* exec_kernel(int vw) {
  if constexpr (sizeof(T) == 8) {
    if (vw == 2) return (const void*)k_exec<T, D, 2, CHAIN, NTS>;
    return (const void*)k_exec<T, D, 1, CHAIN, NTS>;
  } else {
    if (vw == 4) return (const void*)k_exec<T, D, 4, CHAIN, NTS>;
    if (vw == 2) return (const void*)k_exec<T, D, 2, CHAIN, NTS>;
    return (const void*)k_exec<T, D, 1, CHAIN, NTS>;
  }
}

template <typename T, int D, bool CHAIN, int MAXC>
const void* pipe_kernel(int vw) {
  if constexpr (sizeof(T) == 8) {
    if (vw == 2) return (const void*)k_pipe<T, D, 2, CHAIN, MAXC>;
    return (const void*)k_pipe<T, D, 1, CHAIN, MAXC>;
  } else {
    if (vw == 4) return (const void*)k_pipe<T, D, 4, CHAIN, MAXC>;
    if (vw == 2) return (const void*)k_pipe<T, D, 2, CHAIN, MAXC>;
    return (const void*)k_pipe<T, D, 1, CHAIN, MAXC>;
  }
}

// kind: 1 direct-LDS one-shot, 2 register-prefetch persistent (maxc = 8 or
// 16), 3 register one-shot, 4 direct-LDS double-buffered persistent,
// 5 index-pair form (direct-LDS one-shot)
template <typename T, int D>
const void* pick_d(int kind, int vw, bool chain, bool nts, int maxc) {
  if (kind == 5) {
    if (chain) return nts ? (const void*)k_pair<T, D, true, true> : (const void*)k_pair<T, D, true, false>;
    return nts ? (const void*)k_pair<T, D, false, true> : (const void*)k_pair<T, D, false, false>;
  }
  if (kind == 1) {
    if (chain) return nts ? (const void*)k_lds<T, D, true, true> : (const void*)k_lds<T, D, true, false>;
    return nts ? (const void*)k_lds<T, D, false, true> : (const void*)k_lds<T, D, false, false>;
  }
  if (kind == 4) {
    if (chain) return nts ? (const void*)k_ldsp<T, D, true, true> : (const void*)k_ldsp<T, D, true, false>;
    return nts ? (const void*)k_ldsp<T, D, false, true> : (const void*)k_ldsp<T, D, false, false>;
  }
  if (kind == 2) {
    if (maxc == 8) return chain ? pipe_kernel<T, D, true, 8>(vw) : pipe_kernel<T, D, false, 8>(vw);
    return chain ? pipe_kernel<T, D, true, 16>(vw) : pipe_kernel<T, D, false, 16>(vw);
  }
  if (chain) return nts ? exec_kernel<T, D, true, true>(vw) : exec_kernel<T, D, true, false>(vw);
  return nts ? exec_kernel<T, D, false, true>(vw) : exec_kernel<T, D, false, false>(vw);
}

template <typename T, int D>
const void* cgrad_kernel(bool split) {
  if constexpr (D <= 3) {
    if (split) return (const void*)k_cgrad_split<T, D>;
  }
  return (const void*)k_cgrad<T, D>;
}

template <typename T, int D>
const void* pack_kernel(bool pack, bool nts, bool persist) {
  if (pack) return (const void*)k_pack<T, D>;
  if (persist) {
    // (d <= 3 only: a 4D orbit's 24 slots per unit would not stay in registers)
    if constexpr (D <= 3)
      return nts ? (const void*)k_unpack_persist<T, D, true> : (const void*)k_unpack_persist<T, D, false>;
    return nullptr;
  }
  return nts ? (const void*)k_unpack<T, D, true> : (const void*)k_unpack<T, D, false>;
}

template <typename T, int D, bool PERSIST>
const void* batched_kernel_p(int vw) {
  if constexpr (sizeof(T) == 8) {
    if (vw == 2) return (const void*)k_batched<T, D, 2, PERSIST>;
    return (const void*)k_batched<T, D, 1, PERSIST>;
  } else {
    if (vw == 4) return (const void*)k_batched<T, D, 4, PERSIST>;
    if (vw == 2) return (const void*)k_batched<T, D, 2, PERSIST>;
    return (const void*)k_batched<T, D, 1, PERSIST>;
  }
}

template <typename T, int D>
const void* batched_kernel(int vw, bool persist) {
  return persist ? batched_kernel_p<T, D, true>(vw) : batched_kernel_p<T, D, false>(vw);
}

}  // namespace

// Kernel selection, one definition per (storage type, group size) in
// spinsum_kern_<type>_d<d>.hip.
#define SPINSUM_DECLARE_PICK(tag, d)                                                    \
  const void* pick_##tag##_d##d(int kind, int vw, bool chain, bool nts, int maxc);     \
  const void* pick_batched_##tag##_d##d(int vw, bool persist);                         \
  const void* pick_cgrad_##tag##_d##d(bool split);                                      \
  const void* pick_pack_##tag##_d##d(bool pack, bool nts, bool persist);
SPINSUM_DECLARE_PICK(f64, 2)
SPINSUM_DECLARE_PICK(f64, 3)
SPINSUM_DECLARE_PICK(f64, 4)
SPINSUM_DECLARE_PICK(f32, 2)
SPINSUM_DECLARE_PICK(f32, 3)
SPINSUM_DECLARE_PICK(f32, 4)
#undef SPINSUM_DECLARE_PICK

}  // namespace spinsum
