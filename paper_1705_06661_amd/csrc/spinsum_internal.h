// spinsum_internal.h -- data layout shared by the host planner and the gfx950
// kernels of libspinsum.  Not part of the public C-ABI (include/spinsum.h).
//
// Work decomposition (the GPU form of the blocked schedule of Alg. 5a/5b):
//   * the permuted group of every spectator "cube" (N^d contiguous elements,
//     the group being the trailing d dimensions) is cut into tiles by the
//     same partition of [0,N) on every axis (block edge bl, Sec. 4.5);
//   * a tile orbit is the set of tiles {sigma . B : sigma in S_d} of one
//     sorted block tuple B (the b1 <= b2 <= ... loop bounds of Alg. 5a);
//     one workgroup owns one (cube, tile orbit) pair, so every element is
//     read and written by exactly one workgroup -- this ownership is what
//     makes the in-place form (Sec. 4.6.5) safe;
//   * inside the workgroup every element orbit {sigma . x} is combined in
//     registers: with v_sigma = A[sigma . x] the outputs are
//     w_tau = B[tau . x] = sum_sigma M[tau][sigma] v_sigma, where
//     M[tau][sigma] = a(tau^-1 o sigma) and a() is the coefficient of each
//     permutation in the (expanded) operator -- Alg. 2's d! update
//     statements of one element orbit, written as one d! x d! product.
//
// Index-pair form ([.., V x d partner dims, N x d group, inner..], the same
// permutation applied to both index sets): the pair (a_m, i_m) of axis m
// acts as one combined index, and a tile as one combined block
// c_m = a_m * nb + b_m (partner index a_m, group block b_m).  The tile orbits
// are the multisets of d combined blocks; the kernel obtains its orbit by
// reading its sorted combined blocks from a table (8 bytes per orbit,
// against at least 8 * bl^d bytes of data per orbit) and builds the orbit's
// tile list itself.
#pragma once
#include <stdint.h>

#include <utility>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace spinsum {

constexpr int kMaxD = 4;
constexpr int kMaxDF = 24;          // 4!
constexpr int kMaxLdsBytes = 163840; // 160 KiB per CU on gfx950

// Exact division of 0 <= n < 2^31 by a runtime constant (multiply-high
// method, Granlund & Montgomery 1994).
struct FastDiv {
  uint32_t div;
  uint32_t mul;
  uint32_t shift;
  uint32_t pad;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{};
  f.div = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.shift = s;
  f.mul = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
  return f;
}

constexpr int kGradSlots = 2048;     // partial sums of the coefficient gradient (power of 2)
// k_cgrad_split: tiles of an item (a 3D tile orbit at most), element orbits
// per thread, and its workgroup size
constexpr int kCgSplitTiles = 6;
constexpr int kCgSplitUnits = 2;
constexpr int kCgSplitThreads = 256;
constexpr int kUnpackCubeUnits = 6;  // k_unpack_persist: element orbits per thread
constexpr int kUnpackTemplates = 8;  // k_unpack_persist: item templates of a launch
constexpr int kMaxGroupTiles = 24;   // tiles of one work item
constexpr int kMaxGroupOrbits = 8;   // tile orbits of one work item

// One work item template of a cube: a group of tile orbits {sigma . B_k}
// whose tiles sit side by side in LDS (orbit k's tiles after those of
// orbits 0..k-1).  Grouping small orbits (the diagonal ones hold 1 tile, a
// generic 3D one 6) evens the bytes each workgroup moves.
struct alignas(16) GroupDev {
  int32_t ntiles;     // tiles of all orbits of the group
  int32_t norb;       // orbits in the group
  int32_t ragged;     // 1 if some tile is cut by the cube edge
  int32_t rep_total;  // representatives of all orbits of the group
  int32_t tile_off[kMaxGroupTiles];  // element offset of each tile origin inside the cube
  int32_t tile_ext[kMaxGroupTiles];  // extents of each tile, 8 bits per axis (axis 0 lowest)
  int32_t rep_off[kMaxGroupOrbits];  // first representative of orbit k in the pool
  int32_t rep_cnt[kMaxGroupOrbits];  // representatives of orbit k
  int32_t rep_base[kMaxGroupOrbits]; // prefix sum of rep_cnt
  FastDiv fd_rep[kMaxGroupOrbits];   // / rep_cnt[k]
  int32_t slot_base[kMaxGroupOrbits][kMaxDF];  // LDS element offset of tile sigma . B_k
  int32_t eqmask[kMaxGroupOrbits];   // bit m: blocks m and m+1 of B_k are equal
};

// Geometry of one tensor (or one block of a batch).
// A "cube" is the N^d group block of one outer spectator index, each group
// element being a contiguous run of `inner` elements (the inner spectators,
// 1 when the group is trailing).
struct alignas(16) Geom {
  int64_t cube_elems;  // N^d * inner
  int64_t ncubes;      // outer spectator cubes
  int32_t n;           // group extent N
  int32_t bl;          // tile edge
  int32_t ngroups;     // work items (groups of tile orbits) per cube
  int32_t cpw;         // cubes per workgroup (whole-cube mode), else 1
  int32_t gst[kMaxD];  // element strides of the group axes inside a cube
  int32_t lst[kMaxD];  // LDS strides of a tile (padded)
  int32_t ts;          // LDS elements per tile slot
  int32_t cube_lds;    // LDS elements per cube in whole-cube mode
  int32_t rows;        // bl^(d-1) rows per tile
  int32_t vpr;         // vectors per row, bl * inner / VW
  int32_t inner;       // inner spectator run per group element
  int32_t pad0;
  FastDiv fd_vpr;      // / vpr
  FastDiv fd_rows;     // / rows
  FastDiv fd_bl;       // / bl
  FastDiv fd_ngroups;  // / ngroups
  FastDiv fd_inner;    // / inner
};

// One item of a batched launch: a run of whole cubes, or one tile orbit of
// one cube, of one block.
struct alignas(16) BatchItem {
  int64_t cube0;
  int32_t block;
  int32_t group;   // global index into the group pool
  int32_t ncubes;
  int32_t pad;
};

struct alignas(16) BatchBlock {
  Geom g;
  int32_t group_base;
  int32_t pad[3];
};

// Index-pair form: geometry beyond Geom (whose cube is one pair block of
// V^d N^d inner elements, its group strides gst those of the N^d group).
constexpr int kPairKeys = 1 << (2 * kMaxD - 1);  // (equal-neighbour mask, last-block mask)
struct alignas(16) PairGeom {
  int64_t pstride[kMaxD];  // element stride of partner axis m inside a pair block
  int64_t norb;            // tile orbits per pair block: multisets of d combined blocks
                           // (sorted combined blocks of orbit o: 16 bits each in table[o])
  int32_t nc;              // combined blocks per axis, V * nb
  int32_t nb;              // tile blocks per group axis
  int32_t last_ext;        // extent of the last block of a group axis (bl if N % bl == 0)
  int32_t flat;            // 1: bl == N, every tile is one contiguous group cube
  int32_t tile_stride;     // LDS elements per tile slot (flat: plus the alignment shift)
  int32_t pad;
  FastDiv fd_nb;           // / nb
  FastDiv fd_norb;         // / norb (norb < 2^31)
  int32_t rep_off[kPairKeys];  // representative list of each key in the pool
  int32_t rep_cnt[kPairKeys];
};



// ------------------------------------------------------------------------
// Index arithmetic shared by the kernels and by the host-side checker of the
// work decomposition (spinsum_plan_check_ownership), so that the checker
// exercises exactly the addresses the kernels compute.

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
#ifdef __HIP_DEVICE_COMPILE__
  return (__umulhi(n, f.mul) + n) >> f.shift;
#else
  return ((uint32_t)(((uint64_t)n * f.mul) >> 32) + n) >> f.shift;
#endif
}

// Element m of the r-th permutation of (0..d-1) in lexicographic order.
__host__ __device__ constexpr int lex_perm(int d, int r, int m) {
  int avail[4] = {0, 1, 2, 3};
  int navail = d;
  int f = 1;
  for (int k = 2; k < d; ++k) f *= k;
  int res = 0;
  for (int pos = 0; pos < d; ++pos) {
    int idx = r / f;
    r = r % f;
    int val = avail[idx];
    for (int j = idx; j < navail - 1; ++j) avail[j] = avail[j + 1];
    --navail;
    if (pos == m) res = val;
    if (d - 1 - pos > 0) f = f / (d - 1 - pos);
  }
  return res;
}

// Lexicographic rank of a permutation q of (0..d-1) (Lehmer code).
__host__ __device__ constexpr int lex_rank(int d, const int* q) {
  int r = 0;
  for (int m = 0; m < d; ++m) {
    int smaller = 0;
    for (int j = m + 1; j < d; ++j) smaller += (q[j] < q[m]) ? 1 : 0;
    int f = 1;
    for (int k = 2; k <= d - 1 - m; ++k) f *= k;
    r += smaller * f;
  }
  return r;
}

// Rank of tau^-1 o sigma, where (a o b)[m] = a[b[m]] is "operator a applied
// after operator b".  With v_sigma = In[sigma . x] the outputs of an element
// orbit are w_tau = sum_sigma a(tau^-1 o sigma) v_sigma, a() being the
// coefficient of each permutation in the operator.
__host__ __device__ constexpr int ginv_mul(int d, int t, int s) {
  int pt[4] = {0, 0, 0, 0}, inv[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
  for (int m = 0; m < d; ++m) pt[m] = lex_perm(d, t, m);
  for (int m = 0; m < d; ++m) inv[pt[m]] = m;
  for (int m = 0; m < d; ++m) c[m] = inv[lex_perm(d, s, m)];
  return lex_rank(d, c);
}

// Rank of t o p ((a o b)[m] = a[b[m]]): with v_sigma = In[sigma . x], the
// term with permutation p reads v_(tau o p) for the output at tau . x.
__host__ __device__ constexpr int compose(int d, int t, int p) {
  int c[4] = {0, 0, 0, 0};
  for (int m = 0; m < d; ++m) c[m] = lex_perm(d, t, lex_perm(d, p, m));
  return lex_rank(d, c);
}

// Chunk c of a work item (one VW-vector of one tile row) -> global element
// offset from the item's first cube (32 bits: an item spans less than 2^31
// bytes) and LDS element offset; false if the chunk lies outside a ragged
// tile.  toff/text: tile origins and packed extents of the item's orbit.
// A tile row is bl * inner contiguous elements (bl group positions along
// the last group axis, each a run of `inner` elements); l[D-1] is the
// chunk's first element inside its row.
template <int D, int VW>
__host__ __device__ inline bool chunk_addr(const Geom& g, uint32_t c, int ntiles,
                                           const int32_t* toff, const int32_t* text,
                                           bool ragged, int* goff, int* loff) {
  uint32_t q = fdiv(c, g.fd_vpr);
  int v = (int)(c - q * (uint32_t)g.vpr);
  uint32_t q2 = fdiv(q, g.fd_rows);
  int row = (int)(q - q2 * (uint32_t)g.rows);
  int s = (ntiles == 1) ? 0 : (int)q2;
  int cube_i = (ntiles == 1) ? (int)q2 : 0;
  int l[D];
  l[D - 1] = v * VW;
  if constexpr (D == 2) {
    l[0] = row;
  } else {
    uint32_t r = (uint32_t)row;
#pragma unroll
    for (int m = D - 2; m >= 1; --m) {
      uint32_t qq = fdiv(r, g.fd_bl);
      l[m] = (int)(r - qq * (uint32_t)g.bl);
      r = qq;
    }
    l[0] = (int)r;
  }
  bool ok = true;
  if (ragged) {
    int ext = text[s];
#pragma unroll
    for (int m = 0; m < D - 1; ++m) ok = ok && (l[m] < ((ext >> (8 * m)) & 255));
    ok = ok && (l[D - 1] < ((ext >> (8 * (D - 1))) & 255) * g.inner);
  }
  int go = toff[s] + l[D - 1];
  int lo = s * g.ts + l[D - 1];
#pragma unroll
  for (int m = 0; m < D - 1; ++m) {
    go += l[m] * g.gst[m];
    lo += l[m] * g.lst[m];
  }
  *goff = cube_i * (int)g.cube_elems + go;
  *loff = cube_i * g.cube_lds + lo;
  return ok;
}

// Compile-time tables of S_d: element m of permutation r, and the rank of
// r^-1 o s (template constants, so that unrolled kernel code indexes
// registers with literals).
template <int D, int R, int M>
struct LexPerm {
  static constexpr int value = lex_perm(D, R, M);
};
template <int D, int T, int S>
struct GinvMul {
  static constexpr int value = ginv_mul(D, T, S);
};
template <int D, int T, int P>
struct Compose {
  static constexpr int value = compose(D, T, P);
};

// LDS element offset of sigma_R . x for representative x = l[] of a cube
// whose LDS image starts at `base` (combine phase; base includes the inner
// spectator index, lst[d-1] = inner).
template <int D, int R, int... M>
__host__ __device__ inline int orbit_addr_one(const Geom& g, int base, int32_t slot_base_r,
                                              const int* l, std::integer_sequence<int, M...>) {
  return base + slot_base_r + ((l[LexPerm<D, R, M>::value] * g.lst[M]) + ... + 0);
}

// Offsets of sigma . x for every sigma in S_d (lexicographic order).
template <int D, int... R>
__host__ __device__ inline void orbit_addrs(const Geom& g, int base, const int32_t* slot_base,
                                            const int* l, int* addr,
                                            std::integer_sequence<int, R...>) {
  ((addr[R] = orbit_addr_one<D, R>(g, base, slot_base[R], l, std::make_integer_sequence<int, D>{})),
   ...);
}

// Number of non-decreasing L-tuples over m values, C(m + L - 1, L), or -1
// if it exceeds 2^62.
inline int64_t multiset_count(int64_t m, int L) {
  if (L == 0) return 1;
  if (m <= 0) return 0;
  const int64_t x = m + L - 1;
  int64_t r = 1;
  for (int k = 0; k < L; ++k) {
    if (r > ((int64_t)1 << 62) / (x - k)) return -1;
    r = r * (x - k) / (k + 1);  // C(x, k + 1), exact
  }
  return r;
}

// Origin (element offset inside the pair block) and packed extents of the
// tile with combined blocks t[0..d-1].
__host__ __device__ inline void pair_tile(const Geom& g, const PairGeom& pg, int d, const int* t,
                                          int64_t* off, int32_t* ext) {
  int64_t o = 0;
  int32_t e = 0;
  for (int m = 0; m < d; ++m) {
    const int a = (int)fdiv((uint32_t)t[m], pg.fd_nb);
    const int b = t[m] - a * pg.nb;
    o += (int64_t)a * pg.pstride[m] + (int64_t)b * g.bl * g.gst[m];
    e |= ((b == pg.nb - 1) ? pg.last_ext : g.bl) << (8 * m);
  }
  *off = o;
  *ext = e;
}

// Key of the representative list of the orbit with sorted combined blocks
// c: bit m (m < d-1) if c[m] == c[m+1]; bit d-1+m if c[m] is a ragged last
// block.
__host__ __device__ inline int pair_key(const Geom& g, const PairGeom& pg, int d, const int* c) {
  int k = 0;
  for (int m = 0; m + 1 < d; ++m) k |= (c[m] == c[m + 1]) ? (1 << m) : 0;
  for (int m = 0; m < d; ++m) {
    const int a = (int)fdiv((uint32_t)c[m], pg.fd_nb);
    const int b = c[m] - a * pg.nb;
    if (b == pg.nb - 1 && pg.last_ext != g.bl) k |= 1 << (d - 1 + m);
  }
  return k;
}

}  // namespace spinsum
