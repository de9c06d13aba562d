// spinsum_plan.cpp -- host planner of libspinsum: argument validation,
// canonicalisation of the coefficient sets, the group-algebra product of a
// factorised chain (Def. 4), the orbit matrices, the tile-orbit tables of the
// blocked schedule (Alg. 5a/5b) and their upload to the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <utility>

#include "spinsum_plan_host.h"

using spinsum::BatchBlock;
using spinsum::BatchItem;
using spinsum::Geom;
using spinsum::GroupDev;
using spinsum::OrbitHost;
using spinsum::PairGeom;
using spinsum::Tiling;

namespace spinsum {

template <int D>
constexpr int Fact() {
  return D <= 1 ? 1 : D * Fact<(D > 1 ? D - 1 : 1)>();
}

// ------------------------------------------------------------- S_d algebra
void SymGroup::init(int d_) {
  d = d_;
  p.clear();
  std::vector<int> q(d);
  std::iota(q.begin(), q.end(), 0);
  do {
    p.push_back(q);
  } while (std::next_permutation(q.begin(), q.end()));
  df = (int)p.size();
  inv.assign(df, 0);
  mul.assign((size_t)df * df, 0);
  std::vector<int> t(d);
  for (int a = 0; a < df; ++a) {
    for (int m = 0; m < d; ++m) t[p[a][m]] = m;
    inv[a] = rank(t.data());
  }
  for (int a = 0; a < df; ++a)
    for (int b = 0; b < df; ++b) {
      // operator a applied after operator b reads position m -> a[b[m]]
      for (int m = 0; m < d; ++m) t[m] = p[a][p[b][m]];
      mul[(size_t)a * df + b] = rank(t.data());
    }
}

int SymGroup::rank(const int* q) const {
  // Lehmer code in the factorial number system = lexicographic rank
  int r = 0;
  for (int m = 0; m < d; ++m) {
    int smaller = 0;
    for (int j = m + 1; j < d; ++j) smaller += (q[j] < q[m]);
    int f = 1;
    for (int k = 2; k <= d - 1 - m; ++k) f *= k;
    r += smaller * f;
  }
  return r;
}

int elem_size(const spinsum_plan_s& P) { return P.dtype == SPINSUM_F32 ? 4 : 8; }

static int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int k = 0; k < e; ++k) r *= b;
  return r;
}

// Widest vector (elements, at most 16 bytes) dividing a cube row of `row`
// elements (N * inner).
int max_vector_width(const spinsum_plan_s& P, int64_t row) {
  int v = 16 / elem_size(P);
  while (v > 1 && (row % v) != 0) v /= 2;
  return v;
}

// Widest vector dividing both the cube row (n * inner elements) and the tile
// row (bl * inner elements).
static int vw_for(int64_t n_row, int64_t bl_row, int vmax) {
  int v = vmax;
  while (v > 1 && ((n_row % v) != 0 || (bl_row % v) != 0)) v /= 2;
  return v;
}

// LDS strides of a tile: the last group axis has stride `inner` (each group
// position holds a run of inner spectator elements), rows padded by one
// element when pad is set.
static void lds_strides(int d, int bl, int pad, int inner, int32_t* lst, int32_t* ts) {
  lst[d - 1] = inner;
  for (int m = d - 2; m >= 0; --m) {
    int64_t s = (int64_t)lst[m + 1] * bl;
    if (pad && (s % 2) == 0) s += 1;
    lst[m] = (int32_t)s;
  }
  for (int m = d; m < kMaxD; ++m) lst[m] = 0;
  int64_t t = (int64_t)lst[0] * bl;
  if (pad && (t % 2) == 0) t += 1;
  *ts = (int32_t)t;
}

// Largest number of distinct tiles in one orbit for nb blocks per axis.
static int max_orbit_tiles(const SymGroup& G, int nb) {
  const int d = G.d;
  std::vector<int> B(d, 0);
  int best = 0;
  while (true) {
    std::vector<std::vector<int>> tl;
    for (int r = 0; r < G.df; ++r) {
      std::vector<int> t(d);
      for (int m = 0; m < d; ++m) t[m] = B[G.p[r][m]];
      if (std::find(tl.begin(), tl.end(), t) == tl.end()) tl.push_back(t);
    }
    best = std::max(best, (int)tl.size());
    if (best == G.df) break;
    int m = d - 1;
    while (m >= 0 && B[m] == nb - 1) --m;
    if (m < 0) break;
    B[m]++;
    for (int j = m + 1; j < d; ++j) B[j] = B[m];
  }
  return best;
}

// Element orbits of a whole N^d cube under the plan's group (Burnside: the
// mean over the group of N^(cycles of the permutation)).
static int64_t cube_orbits(const SymGroup& G, int n) {
  int64_t sum = 0;
  for (int r = 0; r < G.df; ++r) {
    int cycles = 0;
    bool seen[kMaxD] = {false, false, false, false};
    for (int m = 0; m < G.d; ++m) {
      if (seen[m]) continue;
      ++cycles;
      for (int j = m; !seen[j]; j = G.p[r][j]) seen[j] = true;
    }
    sum += ipow(n, cycles);
  }
  return sum / G.df;
}

static int64_t tile_lds_bytes(const spinsum_plan_s& P, int n, int bl, int cpw, int pad) {
  int32_t lst[kMaxD], ts;
  lds_strides(P.d, bl, pad, P.inner, lst, &ts);
  int nb = (n + bl - 1) / bl;
  int tiles = (bl == n) ? cpw : max_orbit_tiles(P.G, nb);
  // plus the representative copy of the pipelined kernel (at most bl^d)
  return (int64_t)tiles * ts * elem_size(P) + ipow(bl, P.d) * 4;
}

// LDS bank cost of a representative list: the combine step gives the
// representatives to the lanes of a wave in list order (64 per wave), and
// each lane reads and writes element sigma . l of every tile slot sigma,
// at LDS word offset sum_m l[p_sigma(m)] * lst[m] (the slot base is uniform
// across the wave).  The cost sums, over waves and permutations, the largest
// number of distinct 4-byte words that fall in one bank (64 banks, and 32
// as a second model).  The tile slot base adds the same offset to every lane,
// so it does not change the count.
static int64_t rep_bank_cost(const uint32_t* reps, size_t cnt, const SymGroup& G,
                             const int32_t* lst, int esz) {
  const int d = G.d;
  const int words = esz / 4;
  int64_t cost = 0;
  std::vector<uint32_t> w;
  for (size_t g0 = 0; g0 < cnt; g0 += 64) {
    const size_t g1 = std::min(cnt, g0 + 64);
    for (int r = 0; r < G.df; ++r) {
      w.clear();
      for (size_t i = g0; i < g1; ++i) {
        int64_t a = 0;
        for (int m = 0; m < d; ++m) a += (int64_t)((reps[i] >> (8 * G.p[r][m])) & 255u) * lst[m];
        for (int k = 0; k < words; ++k) w.push_back((uint32_t)(a * words + k));
      }
      std::sort(w.begin(), w.end());
      w.erase(std::unique(w.begin(), w.end()), w.end());
      for (int banks : {64, 32}) {
        int hist[64] = {0};
        int worst = 0;
        for (uint32_t x : w) worst = std::max(worst, ++hist[x % banks]);
        cost += worst;
      }
    }
  }
  return cost;
}

// Order the representative list reps[off, end) for the LDS banks.  In
// lexicographic order the 64 lanes of a wave share their leading
// coordinates, so the tile slots that move the fastest axis to a slow one
// make them read words a power of two apart (one 3D 8^3 tile: up to 16
// lanes per bank).  Sorting by the diagonal class (l[d-1] - sum of the
// other coordinates) mod e gives each wave a Latin set instead: for a
// generic list with e^(d-1) = 64, every slot spreads the wave over the
// banks (2 words per bank, the least for 64 lanes of 8 bytes).  The
// order is kept only where the bank cost above drops; every element
// orbit is still combined exactly as before, so results do not change.
static bool order_reps_for_banks(std::vector<uint32_t>& reps, size_t off, const SymGroup& G,
                                 const int32_t* lst, int esz, int e) {
  const int d = G.d;
  const size_t cnt = reps.size() - off;
  if (cnt <= 1 || e <= 1) return false;
  std::vector<uint32_t> alt(reps.begin() + off, reps.end());
  auto cls = [&](uint32_t pk) {
    int c = (int)((pk >> (8 * (d - 1))) & 255u);
    for (int m = 0; m + 1 < d; ++m) c -= (int)((pk >> (8 * m)) & 255u);
    return ((c % e) + e) % e;
  };
  std::stable_sort(alt.begin(), alt.end(),
                   [&](uint32_t x, uint32_t y) { return cls(x) < cls(y); });
  if (rep_bank_cost(alt.data(), cnt, G, lst, esz) >=
      rep_bank_cost(reps.data() + off, cnt, G, lst, esz))
    return false;
  std::copy(alt.begin(), alt.end(), reps.begin() + off);
  return true;
}

// Default tile (measured on MI355X; spinsum_autotune searches more).
//  1. Cubes up to 64 KiB are processed whole, as many per workgroup as
//     make at least 8 KiB, as one contiguous copy (any extent).
//  2. Larger cubes use tile orbits whose rows (also the short rows of
//     ragged edge tiles) are whole 16-byte chunks, for the direct-LDS kernel:
//     rows of at least 32 bytes with the largest orbit within 32 KiB of LDS,
//     else within 64 KiB (large 4D cubes, whose generic orbits have 24
//     tiles), else any such rows within 32 KiB; among the candidates of a
//     pass, the widest rows win, then the smaller LDS footprint.
//  3. Otherwise tiles through registers: the largest whose orbit fits
//     20 KiB of LDS, else the largest that fits.
spinsum_status choose_tile(const spinsum_plan_s& P, int n, int64_t ncubes, int vw,
                           spinsum_tile_t* tile, bool single) {
  const int esz = elem_size(P);
  const int d = P.d;
  const int pad = (P.flags & SPINSUM_FLAG_NO_LDS_PAD) ? 0 : 1;
  const int64_t budget = P.lds_limit - 512;
  spinsum_tile_t t{};
  t.threads = 0;  // chosen once the variant is known
  t.lds_pad = pad;
  const int64_t cube_bytes = ipow(n, d) * P.inner * esz;
  if (cube_bytes <= 64 * 1024 && cube_bytes + 16 + ipow(n, d) * 4 <= budget) {
    t.bl = n;
    // at least 8 KiB per work item: smaller items leave the CU waiting
    // (9^3 FP64 5.84 TB/s with two cubes against 4.33 with one; 11^3 FP32
    // 5.22 with two against 3.41; 9^3 FP32 4.66 with three against 3.79)
    const int64_t cb = std::max<int64_t>(1, cube_bytes);
    int cpw = (int)std::max<int64_t>(1, (8 * 1024 + cb - 1) / cb);
    // keep at least ~8 workgroups per CU of work when the tensor allows it
    int64_t cap = std::max<int64_t>(1, ncubes / (8 * (int64_t)P.num_cus));
    cpw = (int)std::min<int64_t>(cpw, cap);
    t.cubes_per_wg = std::max(1, cpw);
    *tile = t;
    return SPINSUM_OK;
  }
  t.cubes_per_wg = 1;
  struct Pass {
    int min_row;
    int64_t cap;
  };
  const Pass passes[] = {{32, 32 * 1024}, {32, 64 * 1024}, {16, 32 * 1024}};
  int found[3] = {0, 0, 0};
  for (int pi = 0; pi < 3; ++pi) {
    const Pass& ps = passes[pi];
    int best = 0;
    int64_t best_lds = 0;
    for (int bl = n - 1; bl >= 1; --bl) {
      if (bl > 255) continue;
      const int64_t row = (int64_t)bl * P.inner * esz;
      if (row < ps.min_row || vw_for((int64_t)n * P.inner, (int64_t)bl * P.inner, vw) * esz != 16)
        continue;
      const int64_t lb = tile_lds_bytes(P, n, bl, 1, 0);
      if (lb > std::min(ps.cap, budget)) continue;
      if (best == 0 || bl > best || (bl == best && lb < best_lds)) {
        best = bl;
        best_lds = lb;
      }
    }
    found[pi] = best;
  }
  // Rows shorter than half a 128-byte line lose more than the workgroup
  // slots of a larger tile when a tile with two blocks per axis and wider
  // rows lets two workgroups onto a CU (single tensors only).  Its tile
  // orbits are the d + 1 classes by number of upper blocks, and
  // neighbouring classes share every group row: items of consecutive
  // classes up to max(largest class, 1 + d) tiles keep many rows whole in
  // one workgroup.  Measured: 4D 12^4 FP64 (48- instead of 32-byte rows)
  // 4.82 against 4.08 TB/s; 3D 32^3 FP32 (64 instead of 32) 4.80 against
  // 4.39 TB/s.  With 64-byte rows already (3D 24^3 FP64) the wider tile is
  // slower (4.90 against 5.40), so it is not considered there.
  int first = 0;
  for (int pi = 0; pi < 3 && first == 0; ++pi) first = found[pi];
  // Whole cubes of up to a CU's LDS (one workgroup per CU, d <= 3) where
  // the tiles would be slow:
  //  - no tile edge gives rows of whole 16-byte chunks (the register path:
  //    25^3 FP64 0.51 against 5.17 TB/s whole, 30^3 FP32 0.53 against 4.53);
  //  - the tiles are ragged (22^3 / 26^3 FP64 in place 4.71 / 4.24 against
  //    5.03 / 4.77, out of place 2.13 / 2.11 against 4.96 / 4.78; 28^3 FP32
  //    out of place 3.04 against 4.69);
  //  - out of place, FP64 rows shorter than a 128-byte line: nothing has
  //    read the output lines into the L2, so partial rows from different
  //    workgroups reach HBM as partial writes (24^3 5.21 against 4.87).
  // In place, full-sized 64-byte tile rows stay faster (24^3 FP64: 5.41
  // against 5.24), and so do FP32 32^3 cubes out of place (5.00 against
  // 4.17).
  if (single && d <= 3 && cube_bytes + 16 + cube_orbits(P.G, n) * 4 <= budget &&
      (first == 0 || n % first != 0 ||
       (!P.inplace && esz == 8 && (int64_t)first * P.inner * esz < 128))) {
    t.bl = n;
    t.cubes_per_wg = 1;
    *tile = t;
    return SPINSUM_OK;
  }
  if (single && first > 0 && (int64_t)first * P.inner * esz < 64) {
    const int cap = std::max((d == 4) ? 6 : (d == 3) ? 3 : 2, 1 + d);  // C(d, d/2) vs 1 + d
    for (int bl = std::min(n - 1, 255); bl > first && (n + bl - 1) / bl <= 2; --bl) {
      if (vw_for((int64_t)n * P.inner, (int64_t)bl * P.inner, vw) * esz != 16) continue;
      int32_t lst[kMaxD], ts;
      lds_strides(d, bl, 0, P.inner, lst, &ts);
      const int64_t lb = (int64_t)cap * ts * esz + ipow(bl, d) * 4;
      if (lb > std::min<int64_t>(P.lds_limit / 2, budget)) continue;
      t.bl = bl;
      t.item_tiles = cap;
      *tile = t;
      return SPINSUM_OK;
    }
  }
  for (int pi = 0; pi < 3; ++pi)
    if (found[pi] > 0) {
      t.bl = found[pi];
      *tile = t;
      return SPINSUM_OK;
    }
  // The register path: small tile orbits first, so that many workgroups
  // share a CU (measured: 33^3 FP64 2.96 TB/s at bl = 7 with 16 KiB of LDS
  // against 0.93 at bl = 17 with 115 KiB; 37^3 FP32 1.42 at bl = 7 against
  // 0.35 at bl = 21), then the largest that fits.
  for (const int64_t cap : {(int64_t)20 * 1024, budget}) {
    for (int bl = n - 1; bl >= 1; --bl) {
      if (bl > 255) continue;
      if (vw > 1 && ((int64_t)bl * P.inner) % vw != 0) continue;
      if (tile_lds_bytes(P, n, bl, 1, pad) > std::min(cap, budget)) continue;
      t.bl = bl;
      *tile = t;
      return SPINSUM_OK;
    }
  }
  return SPINSUM_ERR_UNSUPPORTED;
}

spinsum_status build_tiling(const spinsum_plan_s& P, int n, int64_t ncubes,
                            const spinsum_tile_t& tile, int vmax, Tiling* out) {
  const SymGroup& G = P.G;
  const int d = P.d;
  Tiling T;
  if (n <= 0 || ncubes <= 0) {
    T.g.ncubes = std::max<int64_t>(0, ncubes);
    T.g.n = n;
    T.g.inner = std::max(1, P.inner);
    T.g.fd_inner = make_fastdiv((uint32_t)T.g.inner);
    *out = T;
    return SPINSUM_OK;
  }
  int bl = tile.bl <= 0 ? n : std::min(tile.bl, n);
  if (bl > 255) return SPINSUM_ERR_UNSUPPORTED;
  const int pad = tile.lds_pad ? 1 : 0;
  const int cpw = (bl == n) ? std::max(1, tile.cubes_per_wg) : 1;
  const int inner = P.inner;
  const int64_t cube_elems = ipow(n, d) * inner;
  if (cube_elems * elem_size(P) >= (1ll << 31)) return SPINSUM_ERR_UNSUPPORTED;
  const int nb = (n + bl - 1) / bl;
  const int vw = vw_for((int64_t)n * inner, (int64_t)bl * inner, vmax);

  Geom& g = T.g;
  g.cube_elems = cube_elems;
  g.ncubes = ncubes;
  g.n = n;
  g.bl = bl;
  g.cpw = cpw;
  for (int m = 0; m < kMaxD; ++m) g.gst[m] = 0;
  for (int m = 0; m < d; ++m) g.gst[m] = (int32_t)(ipow(n, d - 1 - m) * inner);
  lds_strides(d, bl, pad, inner, g.lst, &g.ts);
  g.cube_lds = g.ts;
  g.rows = (int32_t)ipow(bl, d - 1);
  g.vpr = bl * inner / vw;
  g.inner = inner;
  g.pad0 = 0;
  g.fd_vpr = make_fastdiv((uint32_t)g.vpr);
  g.fd_rows = make_fastdiv((uint32_t)g.rows);
  g.fd_bl = make_fastdiv((uint32_t)bl);
  g.fd_inner = make_fastdiv((uint32_t)inner);

  // 1. tile orbits: one per sorted block tuple B (the loop nest of Alg. 5a)
  std::map<std::vector<int>, std::pair<int, int>> rep_index;  // shared representative lists
  bool reordered = false;
  std::vector<int> B(d, 0);
  while (true) {
    OrbitHost oh;
    std::vector<std::vector<int>> tl;
    for (int r = 0; r < G.df; ++r) {
      std::vector<int> t(d);
      for (int m = 0; m < d; ++m) t[m] = B[G.p[r][m]];
      auto it = std::find(tl.begin(), tl.end(), t);
      if (it == tl.end()) {
        oh.slot[r] = (int)tl.size();
        tl.push_back(t);
      } else {
        oh.slot[r] = (int)(it - tl.begin());
      }
    }
    oh.ntiles = (int)tl.size();
    for (int m = 0; m < d; ++m) oh.B[m] = B[m];
    for (int s = 0; s < oh.ntiles; ++s) {
      int64_t off = 0;
      int32_t ext = 0;
      for (int m = 0; m < d; ++m) {
        off += (int64_t)tl[s][m] * bl * g.gst[m];
        int e = std::min(bl, n - tl[s][m] * bl);
        if (e < bl) oh.ragged = 1;
        ext |= (e & 255) << (8 * m);
      }
      oh.tile_off[s] = (int32_t)off;
      oh.tile_ext[s] = ext;
    }
    // canonical representatives: inside tile B, sorted within runs of equal blocks
    std::vector<int> key;
    int extB[kMaxD];
    for (int m = 0; m < d; ++m) {
      extB[m] = std::min(bl, n - B[m] * bl);
      key.push_back(extB[m]);
    }
    for (int m = 0; m + 1 < d; ++m) key.push_back(B[m] == B[m + 1]);
    auto ri = rep_index.find(key);
    if (ri == rep_index.end()) {
      int off = (int)T.reps.size();
      std::vector<int> l(d, 0);
      int64_t box = 1;
      for (int m = 0; m < d; ++m) box *= extB[m];
      for (int64_t e = 0; e < box; ++e) {
        int64_t rem = e;
        for (int m = d - 1; m >= 0; --m) {
          l[m] = (int)(rem % extB[m]);
          rem /= extB[m];
        }
        bool ok = true;
        for (int m = 0; m + 1 < d; ++m)
          if (B[m] == B[m + 1] && l[m] > l[m + 1]) ok = false;
        if (!ok) continue;
        uint32_t pk = 0;
        for (int m = 0; m < d; ++m) pk |= (uint32_t)l[m] << (8 * m);
        T.reps.push_back(pk);
      }
      T.reps_lex.insert(T.reps_lex.end(), T.reps.begin() + off, T.reps.end());
      if (inner == 1 && order_reps_for_banks(T.reps, (size_t)off, G, g.lst, elem_size(P), bl))
        reordered = true;
      ri = rep_index.emplace(key, std::make_pair(off, (int)T.reps.size() - off)).first;
    }
    oh.rep_off = ri->second.first;
    oh.rep_cnt = ri->second.second;
    T.max_orbit_tiles = std::max(T.max_orbit_tiles, oh.ntiles);
    T.ragged |= oh.ragged;
    T.orbits.push_back(oh);
    int m = d - 1;
    while (m >= 0 && B[m] == nb - 1) --m;
    if (m < 0) break;
    B[m]++;
    for (int j = m + 1; j < d; ++j) B[j] = B[m];
  }

  // Large cubes (more tile orbits than an XCD runs at once): order the
  // orbits by their "line block" tuple.  Tiles whose rows share cache lines
  // along the fastest axis (block b and its neighbours within one line,
  // b / s for s tiles per line) get the same key, so their orbits are
  // neighbours in the item list -- and land on the same XCD, close in time.
  // Within a key, the loop-nest order is kept.  (Measured: +12% for one
  // 352^3 cube; for cubes of a few dozen orbits, which an XCD processes
  // together anyway, the loop-nest order is 2% faster.)
  if (T.orbits.size() > 128) {
    const int line = 128;
    const int64_t row = (int64_t)bl * inner * elem_size(P);
    const int s = (row < line && line % row == 0 && ((int64_t)n * inner * elem_size(P)) % line == 0)
                      ? (int)(line / row)
                      : 1;
    if (s > 1) {
      // Within a line-block tuple, the offsets B[m] mod s follow Morton
      // order (their bits interleaved across the axes, high bits first).
      // Two orbits whose tiles share a line differ in one offset; where
      // they share a 64-byte half line they differ in its lowest bit, and
      // are then at most 2^(d-1) positions apart (s^(d-1) in loop-nest
      // order).
      int sbits = 0;
      while ((1 << sbits) < s) ++sbits;
      auto key = [&](const OrbitHost& o) {
        std::vector<int> k(d + 1);
        for (int m = 0; m < d; ++m) k[m] = o.B[m] / s;
        int z = 0;
        for (int b = sbits - 1; b >= 0; --b)
          for (int m = 0; m < d; ++m) z = (z << 1) | (((o.B[m] % s) >> b) & 1);
        k[d] = z;
        return k;
      };
      std::stable_sort(T.orbits.begin(), T.orbits.end(),
                       [&](const OrbitHost& a, const OrbitHost& b) { return key(a) < key(b); });
    }
  }

  if (!reordered) T.reps_lex.clear();

  // 2. work items: one tile orbit each (item_tiles 0), or runs of
  //    consecutive orbits of the order above (next fit), holding at most
  //    `cap` tiles and kMaxGroupOrbits orbits.  Neighbouring orbits hold the
  //    tiles that share group rows and 128-byte lines (with two blocks per
  //    axis: the orbits with k and k+1 upper blocks), so packing them keeps
  //    those rows within one workgroup.  (Measured against first fit by
  //    decreasing size: 4.82 against 4.46-4.67 TB/s on the 4D 12^4 slab.)
  if (T.max_orbit_tiles > kMaxGroupTiles) return SPINSUM_ERR_UNSUPPORTED;
  const int cap = std::min(std::max(tile.item_tiles, T.max_orbit_tiles), kMaxGroupTiles);
  std::vector<std::vector<int>> bins;
  int fill = 0;
  for (int o = 0; o < (int)T.orbits.size(); ++o) {
    const int nt = T.orbits[o].ntiles;
    if (tile.item_tiles <= 0 || bins.empty() || fill + nt > cap ||
        (int)bins.back().size() >= kMaxGroupOrbits) {
      bins.push_back({});
      fill = 0;
    }
    bins.back().push_back(o);
    fill += nt;
  }
  for (const std::vector<int>& bin : bins) {
    GroupDev gd;
    std::memset(&gd, 0, sizeof(gd));
    int tbase = 0, rbase = 0;
    for (int k = 0; k < (int)bin.size(); ++k) {
      const OrbitHost& oh = T.orbits[bin[k]];
      for (int s = 0; s < oh.ntiles; ++s) {
        gd.tile_off[tbase + s] = oh.tile_off[s];
        gd.tile_ext[tbase + s] = oh.tile_ext[s];
      }
      for (int r = 0; r < G.df; ++r) gd.slot_base[k][r] = (tbase + oh.slot[r]) * g.ts;
      gd.rep_off[k] = oh.rep_off;
      gd.rep_cnt[k] = oh.rep_cnt;
      gd.rep_base[k] = rbase;
      gd.fd_rep[k] = make_fastdiv((uint32_t)std::max(1, oh.rep_cnt));
      for (int m = 0; m + 1 < d; ++m)
        if (oh.B[m] == oh.B[m + 1]) gd.eqmask[k] |= 1 << m;
      gd.ragged |= oh.ragged;
      tbase += oh.ntiles;
      rbase += oh.rep_cnt;
    }
    gd.ntiles = tbase;
    gd.norb = (int)bin.size();
    gd.rep_total = rbase;
    T.max_tiles = std::max(T.max_tiles, tbase);
    T.max_rep_cnt = std::max(T.max_rep_cnt, rbase);
    T.groups.push_back(gd);
  }
  g.ngroups = (int32_t)T.groups.size();
  g.fd_ngroups = make_fastdiv((uint32_t)g.ngroups);
  T.nb = nb;
  T.vw = vw;
  // whole cubes: plus one 16-byte chunk for the alignment shift of the
  // contiguous copy
  T.lds_elems = (bl == n) ? (int64_t)cpw * g.ts + 16 / elem_size(P) : (int64_t)T.max_tiles * g.ts;
  T.nitems = (bl == n) ? (ncubes + cpw - 1) / cpw : ncubes * g.ngroups;
  {
    int64_t chunks = (int64_t)((bl == n) ? cpw : T.max_tiles) * g.rows * g.vpr;
    T.chunks_per_thread = (int)((chunks + 255) / 256);
  }
  if ((bl == n) && (int64_t)cpw * cube_elems * elem_size(P) >= (1ll << 31)) return SPINSUM_ERR_UNSUPPORTED;
  // tiles, the representative copy of the pipelined kernel, static tables
  T.fits = ((T.lds_elems * elem_size(P) + 15) / 16 * 16 + (int64_t)T.max_rep_cnt * 4 + 512 <=
            P.lds_limit) ? 1 : 0;
  if (!T.fits && !(P.flags & SPINSUM_FLAG_HOST_ONLY)) return SPINSUM_ERR_UNSUPPORTED;
  if (T.nitems >= (1ll << 31) - 8) return SPINSUM_ERR_UNSUPPORTED;
  *out = std::move(T);
  return SPINSUM_OK;
}

// ------------------------------------------------------------ device tables
static spinsum_status hip_fail(spinsum_plan_s* P, hipError_t e) {
  P->last_hip_error = (int)e;
  return SPINSUM_ERR_HIP;
}

void free_device(spinsum_plan_s* P) {
  void** ptrs[] = {&P->d_orbits,    &P->d_reps,        &P->d_mats,      &P->d_blocks,
                   &P->d_items,     &P->d_grad_part,   &P->d_cg_orbits, &P->d_cg_reps,
                   &P->d_reps_lex,  &P->d_pk_orbits,   &P->d_pk_reps};
  for (void** p : ptrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  P->has_dev = false;
  P->cg_pack = false;
  P->pk_own = false;
}

template <typename V>
static spinsum_status upload(spinsum_plan_s* P, void** dst, const V* src, size_t count) {
  size_t bytes = std::max<size_t>(sizeof(V), count * sizeof(V));
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    P->last_hip_error = (int)e;
    return e == hipErrorOutOfMemory ? SPINSUM_ERR_OUT_OF_MEMORY : SPINSUM_ERR_HIP;
  }
  if (count) {
    e = hipMemcpy(*dst, src, count * sizeof(V), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(P, e);
  }
  return SPINSUM_OK;
}

// The coefficient gradient keeps x and the upstream gradient in LDS, twice
// the tiles of the forward kernel.  Where that lets fewer than four of its
// workgroups onto a CU and the forward tiling has one orbit per item, it
// gets a tiling of its own with consecutive orbits packed up to the largest
// one (3D 32^3 slab: 3.51 -> 4.18 TB/s).
static bool cgrad_split_ok(const spinsum_plan_s& P) {
  const Tiling& T = P.T;
  if (P.pair || P.batched || P.d > 3 || T.g.bl >= T.g.n || T.g.inner != 1) return false;
  if (P.tile.variant != SPINSUM_VARIANT_DIRECT_LDS || P.tile.lds_pad != 0) return false;
  if ((int64_t)T.vw * elem_size(P) != 16) return false;
  if ((int64_t)T.g.rows * T.g.vpr > kCgSplitThreads) return false;
  for (const GroupDev& gd : T.groups)
    if (gd.norb != 1 || gd.ntiles > kCgSplitTiles || gd.rep_cnt[0] > kCgSplitUnits * kCgSplitThreads)
      return false;
  const int64_t lds = (T.lds_elems * elem_size(P) + 15) / 16 * 16 + (int64_t)T.max_rep_cnt * 4;
  return lds <= P.lds_limit;
}

static spinsum_status build_cgrad_tiling(spinsum_plan_s* P) {
  const Tiling& T = P->T;
  const int esz = elem_size(*P);
  if (P->cg_split) return SPINSUM_OK;  // one tile buffer: no packed tiling needed
  auto cg_lds = [&](const Tiling& X) {
    return 2 * ((X.lds_elems * esz + 15) / 16 * 16) + (int64_t)X.max_rep_cnt * 4;
  };
  const int vmax = max_vector_width(*P, (int64_t)std::max(1, P->n) * P->inner);
  if (!P->pair && !P->batched && T.g.bl >= T.g.n && P->tile.lds_pad == 0 &&
      cg_lds(T) > P->lds_limit) {
    // whole cubes too large for both tensors (out of place, FP64 cubes up
    // to a CU's LDS are summed whole): the gradient takes tiles of its own,
    // the largest edge with whole 16-byte chunks per row whose tile orbits,
    // both tensors, fit half a CU's LDS
    for (int bl = P->n - 1; bl >= 1; --bl) {
      spinsum_tile_t t = P->tile;
      t.bl = bl;
      t.cubes_per_wg = 1;
      t.item_tiles = 0;
      t.threads = 0;
      Tiling Tc;
      if (build_tiling(*P, P->n, P->ncubes, t, vmax, &Tc) != SPINSUM_OK) continue;
      if (!Tc.fits || (int64_t)Tc.vw * esz != 16 || cg_lds(Tc) > P->lds_limit / 2) continue;
      spinsum_status st = upload(P, &P->d_cg_orbits, Tc.groups.data(), Tc.groups.size());
      if (st != SPINSUM_OK) return st;
      st = upload(P, &P->d_cg_reps, Tc.reps.data(), Tc.reps.size());
      if (st != SPINSUM_OK) return st;
      P->Tc = std::move(Tc);
      P->cg_pack = true;
      return SPINSUM_OK;
    }
    return SPINSUM_OK;
  }
  if (P->pair || P->batched || T.g.bl >= T.g.n || T.orbits.size() < 2 ||
      T.groups.size() != T.orbits.size() || P->tile.lds_pad != 0)
    return SPINSUM_OK;
  if (P->lds_limit / std::max<int64_t>(1, cg_lds(T)) >= 4) return SPINSUM_OK;
  spinsum_tile_t t = P->tile;
  t.item_tiles = T.max_orbit_tiles;
  Tiling Tc;
  if (build_tiling(*P, P->n, P->ncubes, t, vmax, &Tc) != SPINSUM_OK) return SPINSUM_OK;
  if (cg_lds(Tc) > P->lds_limit || Tc.vw != T.vw) return SPINSUM_OK;
  spinsum_status st = upload(P, &P->d_cg_orbits, Tc.groups.data(), Tc.groups.size());
  if (st != SPINSUM_OK) return st;
  st = upload(P, &P->d_cg_reps, Tc.reps.data(), Tc.reps.size());
  if (st != SPINSUM_OK) return st;
  P->Tc = std::move(Tc);
  P->cg_pack = true;
  return SPINSUM_OK;
}

// Store mode (measured on MI355X): non-temporal stores stream whole lines
// best (3D o=32 slab: +2 %), but where tile rows are shorter than 64 bytes,
// or a cube is cut into more than 128 tile orbits (the items that write the
// parts of one 128-byte line then run far apart), cached stores let the L2
// merge the partial lines first: 4D o=12 slab +3 %, one 352^3 cube +2.5 %,
// one 80^4 cube +10 %.
static int choose_nts(const spinsum_plan_s& P, const Tiling& T, int64_t orbits) {
  if (P.flags & SPINSUM_FLAG_NO_NT_STORES) return 0;
  if (P.flags & SPINSUM_FLAG_NT_STORES) return 1;
  const bool whole = (T.g.bl == T.g.n) && !P.pair;
  if (whole) return 1;
  const int64_t row = (int64_t)T.g.bl * T.g.inner * elem_size(P);
  return (row >= 64 && orbits <= 128) ? 1 : 0;
}

// Load policy of the direct-LDS kernel: non-temporal where every work item
// owns the 128-byte lines it reads, so that no other item needs them in the
// L2 -- whole cubes (one contiguous run per item), or tile rows that start
// and end on line boundaries (the row stride, the tile row and the ragged
// last tile row all multiples of 128 bytes).  Measured on MI355X: inner
// runs of 8 (256-byte rows) +5 %, Fig. 1b's subgroup plan +6 %, whole
// 24^3 FP32 cubes +3 to +4 %; with 64-byte rows the same loads are 14 %
// slower, and with 32-byte rows in one 80^4 cube 23 %.
static int choose_ntl(const spinsum_plan_s& P, const Tiling& T) {
  if (P.flags & SPINSUM_FLAG_NO_NT_LOADS) return 0;
  if (P.pair || T.g.n <= 0) return 0;
  if (T.g.bl == T.g.n) return 1;
  const int64_t e = (int64_t)T.g.inner * elem_size(P);
  const int64_t last = T.g.n - (int64_t)(T.nb - 1) * T.g.bl;
  return ((e * T.g.n) % 128 == 0 && (e * T.g.bl) % 128 == 0 && (e * last) % 128 == 0) ? 1 : 0;
}

// Unpacking's own tiling where it differs from T (pk_own).  Unpacking reads
// only the packed values and writes every element of its items once, so it
// gains from the largest items a CU holds: whole cubes where a cube (with
// its representative list) fits the LDS, else the largest tile edge whose
// rows are whole 128-byte lines and whose items fit.  The sum and packing
// keep T.  Measured on MI355X: whole 24^3 FP64 cubes 4.24 against 2.60
// TB/s, whole 32^3 FP32 cubes 3.37 against 2.46, bl = 16 on 32^3 FP64
// cubes 2.98 against 2.68 (packing with the same tiles: equal, or 27-37 %
// slower).
static void choose_unpack_tiling(spinsum_plan_s* P) {
  P->pk_own = false;
  P->pk_persist = false;
  const Tiling& T = P->T;
  // (whole cubes several to a workgroup keep the plan's items; whole cubes
  // one to a workgroup take the persistent kernel below)
  if (P->pair || P->batched || P->ncubes <= 0 || P->elems <= 0 ||
      (T.g.bl >= T.g.n && T.g.cpw > 1) || P->tile.lds_pad != 0 ||
      P->tile.variant != SPINSUM_VARIANT_DIRECT_LDS)
    return;
  const int esz = elem_size(*P);
  const int d = P->d;
  int64_t df = 1;
  for (int k = 2; k <= d; ++k) df *= k;
  const int vmax = max_vector_width(*P, (int64_t)P->n * P->inner);
  auto lds_of = [&](const Tiling& X) {
    return (X.lds_elems * esz + 15) / 16 * 16 + (int64_t)X.max_rep_cnt * 4;
  };
  std::vector<int> cand;
  if (ipow(P->n, d) * P->inner * esz <= P->lds_limit) cand.push_back(P->n);  // whole cubes
  for (int bl = P->n - 1; bl > T.g.bl; --bl) {
    const int64_t tile_bytes = ipow(bl, d) * P->inner * esz;
    const int nb = (P->n + bl - 1) / bl;
    if (((int64_t)bl * P->inner * esz) % 128 != 0) continue;
    if (tile_bytes * (nb >= d ? df : 1) > P->lds_limit) continue;  // a generic orbit's tiles
    cand.push_back(bl);
  }
  for (int bl : cand) {
    spinsum_tile_t t = P->tile;
    t.bl = bl;
    t.cubes_per_wg = 1;
    t.item_tiles = 0;
    t.threads = 0;
    Tiling Tu;
    if (build_tiling(*P, P->n, P->ncubes, t, vmax, &Tu) != SPINSUM_OK) continue;
    if (!Tu.fits || lds_of(Tu) > P->lds_limit) continue;
    if (bl < P->n && (int64_t)Tu.vw * esz != 16) continue;  // rows of whole 16-byte chunks
    const int64_t per_cu = std::max<int64_t>(1, P->lds_limit / std::max<int64_t>(1, lds_of(Tu)));
    Tu.nts = choose_nts(*P, Tu, (int64_t)Tu.orbits.size());
    P->pk_threads = per_cu >= 4 ? 256 : per_cu >= 2 ? 512 : 1024;
    P->Tu = std::move(Tu);
    P->pk_own = true;
    // items of one tile orbit (or one whole cube) each, of at most
    // kUnpackTemplates templates (d <= 3), whose element orbits the
    // workgroup's threads hold all at once (kUnpackCubeUnits each) and whose
    // packed offsets fit 31 bits: the persistent kernel, k_unpack_persist
    const Tiling& U = P->Tu;
    if (d <= 3 && U.g.cpw == 1 && !U.groups.empty() &&
        (int)U.groups.size() <= kUnpackTemplates) {
      int64_t nc = 1;
      for (int k = 0; k < d; ++k) nc = nc * (P->n - k) / (k + 1);
      bool ok = nc * P->inner < ((int64_t)1 << 31);
      for (const GroupDev& gd : U.groups)
        ok = ok && gd.norb == 1 &&
             (int64_t)gd.rep_cnt[0] * P->inner <= (int64_t)kUnpackCubeUnits * P->pk_threads;
      P->pk_persist = ok;
    }
    return;
  }
}

spinsum_status upload_tables(spinsum_plan_s* P) {
  free_device(P);
  P->cg_split = cgrad_split_ok(*P);
  choose_unpack_tiling(P);
  if (P->flags & SPINSUM_FLAG_HOST_ONLY) return SPINSUM_OK;
  spinsum_status st;
  // coefficient vectors in the storage type: forward | adjoint | stages | adjoint stages
  std::vector<double> all;
  all.insert(all.end(), P->M.begin(), P->M.end());
  all.insert(all.end(), P->MT.begin(), P->MT.end());
  all.insert(all.end(), P->SM.begin(), P->SM.end());
  all.insert(all.end(), P->SMT.begin(), P->SMT.end());
  if (P->dtype == SPINSUM_F32) {
    std::vector<float> f(all.begin(), all.end());
    st = upload(P, &P->d_mats, f.data(), f.size());
  } else {
    st = upload(P, &P->d_mats, all.data(), all.size());
  }
  if (st != SPINSUM_OK) return st;
  if (P->pair) {
    st = upload(P, &P->d_orbits, P->pair_orbits.data(), P->pair_orbits.size());
    if (st != SPINSUM_OK) return st;
    st = upload(P, &P->d_reps, P->T.reps.data(), P->T.reps.size());
    if (st != SPINSUM_OK) return st;
  } else if (!P->batched) {
    st = upload(P, &P->d_orbits, P->T.groups.data(), P->T.groups.size());
    if (st != SPINSUM_OK) return st;
    st = upload(P, &P->d_reps, P->T.reps.data(), P->T.reps.size());
    if (st != SPINSUM_OK) return st;
    if (!P->T.reps_lex.empty()) {
      st = upload(P, &P->d_reps_lex, P->T.reps_lex.data(), P->T.reps_lex.size());
      if (st != SPINSUM_OK) return st;
    }
    std::vector<double> part((size_t)kGradSlots * P->G.df, 0.0);
    st = upload(P, &P->d_grad_part, part.data(), part.size());
    if (st != SPINSUM_OK) return st;
    st = build_cgrad_tiling(P);
    if (st != SPINSUM_OK) return st;
    if (P->pk_own) {
      st = upload(P, &P->d_pk_orbits, P->Tu.groups.data(), P->Tu.groups.size());
      if (st != SPINSUM_OK) return st;
      st = upload(P, &P->d_pk_reps, P->Tu.reps.data(), P->Tu.reps.size());
      if (st != SPINSUM_OK) return st;
    }
  } else {
    std::vector<GroupDev> groups;
    std::vector<uint32_t> reps;
    for (const Tiling& t : P->btil) {
      int roff = (int)reps.size();
      for (GroupDev gd : t.groups) {
        for (int k = 0; k < gd.norb; ++k) gd.rep_off[k] += roff;
        groups.push_back(gd);
      }
      reps.insert(reps.end(), t.reps.begin(), t.reps.end());
    }
    st = upload(P, &P->d_orbits, groups.data(), groups.size());
    if (st != SPINSUM_OK) return st;
    st = upload(P, &P->d_reps, reps.data(), reps.size());
    if (st != SPINSUM_OK) return st;
    st = upload(P, &P->d_blocks, P->blocks.data(), P->blocks.size());
    if (st != SPINSUM_OK) return st;
    st = upload(P, &P->d_items, P->items.data(), P->items.size());
    if (st != SPINSUM_OK) return st;
  }
  P->has_dev = true;
  return cache_occupancy(P);
}

}  // namespace spinsum

using namespace spinsum;

// ------------------------------------------------------------ plan building
static spinsum_status set_terms(spinsum_plan_s* P, int nstages, const int* nterms,
                                const int* perms, const double* alpha) {
  const int d = P->d;
  if (nstages < 1 || nstages > 64 || nterms == nullptr) return SPINSUM_ERR_INVALID_ARG;
  int total = 0;
  for (int k = 0; k < nstages; ++k) {
    if (nterms[k] < 0 || nterms[k] > 1 << 20) return SPINSUM_ERR_INVALID_ARG;
    total += nterms[k];
  }
  if (total > 0 && (perms == nullptr || alpha == nullptr)) return SPINSUM_ERR_INVALID_ARG;
  for (int t = 0; t < total; ++t) {
    bool seen[kMaxD] = {false, false, false, false};
    for (int m = 0; m < d; ++m) {
      int v = perms[t * d + m];
      if (v < 0 || v >= d || seen[v]) return SPINSUM_ERR_NOT_PERMUTATION;
      seen[v] = true;
    }
    if (!std::isfinite(alpha[t])) return SPINSUM_ERR_INVALID_ARG;
  }
  const SymGroup& G = P->G;
  const int df = G.df;
  P->stage_a.assign(nstages, std::vector<double>(df, 0.0));
  int t = 0;
  for (int k = 0; k < nstages; ++k)
    for (int j = 0; j < nterms[k]; ++j, ++t) P->stage_a[k][G.rank(perms + (size_t)t * d)] += alpha[t];
  // expanded operator: E = a_{K-1} * ... * a_0 (later stages act after earlier ones)
  P->expanded = P->stage_a[0];
  for (int k = 1; k < nstages; ++k) {
    std::vector<double> e(df, 0.0);
    for (int a = 0; a < df; ++a) {
      if (P->stage_a[k][a] == 0.0) continue;
      for (int b = 0; b < df; ++b)
        if (P->expanded[b] != 0.0) e[G.mul[(size_t)a * df + b]] += P->stage_a[k][a] * P->expanded[b];
    }
    P->expanded = e;
  }
  // The kernels index the coefficient vector with ginv_mul(); it must agree
  // with the group tables used here.
  for (int t = 0; t < df; ++t)
    for (int sg = 0; sg < df; ++sg)
      if (ginv_mul(P->d, t, sg) != G.mul[(size_t)G.inv[t] * df + sg]) return SPINSUM_ERR_UNSUPPORTED;
  // coefficient vectors: forward (expanded), adjoint a'(g) = a(g^-1), and
  // per stage in application order (forward: stage 0 first; adjoint: last
  // stage first, each inverted)
  auto adjoint_of = [&](const std::vector<double>& a) {
    std::vector<double> r(df);
    for (int g = 0; g < df; ++g) r[g] = a[G.inv[g]];
    return r;
  };
  P->M = P->expanded;
  P->MT = adjoint_of(P->expanded);
  P->SM.clear();
  P->SMT.clear();
  for (int k = 0; k < nstages; ++k) P->SM.insert(P->SM.end(), P->stage_a[k].begin(), P->stage_a[k].end());
  for (int k = nstages - 1; k >= 0; --k) {
    std::vector<double> r = adjoint_of(P->stage_a[k]);
    P->SMT.insert(P->SMT.end(), r.begin(), r.end());
  }
  // Which coefficient vectors leave out a permutation, as the kernels see
  // them (rounded to the storage type): those combine an element orbit
  // term by term once one of its inputs is Inf or NaN (Def. 3 sums only
  // the operator's terms).  Inverting every permutation keeps the zeros'
  // count, so the adjoint vectors share the forward ones' answer.
  auto has_zero = [&](const double* a) {
    for (int g = 0; g < df; ++g) {
      const double c = (P->dtype == SPINSUM_F32) ? (double)(float)a[g] : a[g];
      if (c == 0.0) return true;
    }
    return false;
  };
  P->sparse_expanded = has_zero(P->expanded.data()) ? 1u : 0u;
  P->sparse_fwd = 0;
  P->sparse_adj = 0;
  for (int k = 0; k < nstages; ++k) {  // the kernels treat stages from 32 on as sparse
    if (has_zero(P->stage_a[k].data())) {
      if (k < 32) P->sparse_fwd |= 1u << k;
      if (nstages - 1 - k < 32) P->sparse_adj |= 1u << (nstages - 1 - k);
    }
  }
  return SPINSUM_OK;
}

static void query_device(spinsum_plan_s* P) {
  P->num_cus = 256;
  P->lds_limit = kMaxLdsBytes;
  if (P->flags & SPINSUM_FLAG_HOST_ONLY) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  P->device = dev;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    P->num_cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    P->lds_limit = std::min(v, kMaxLdsBytes);
  (void)hipGetLastError();
}

// ---------------------------------------------------------- index-pair form
// Tensor [outer.., V x d partners, N x d group, inner..], term p applied to
// both index sets.  Axis m carries the pair (a_m, i_m); with the group cut
// into nb blocks of edge bl, a tile is one combined block c_m = a_m * nb + b_m
// per axis: the bl^d group positions of block tuple b under the partner
// tuple a.  A permutation maps tile c to tile sigma . c and element l of it
// to sigma . l, exactly as in the group form, so the tile orbits are the
// multisets of d combined blocks and the element orbits inside a tile are
// those of its equal-block pattern (Alg. 5a/5b on combined indices).

// LDS bytes the index-pair kernel needs for tile edge bl (0 if bl is not
// usable: a partial cube whose rows are not whole 16-byte chunks).
static int64_t pair_lds_bytes(const spinsum_plan_s& P, int bl, int* vw_out) {
  const int n = P.n, d = P.d, esz = elem_size(P), inner = P.inner;
  const bool flat = (bl == n);
  int vw = vw_for((int64_t)n * inner, (int64_t)bl * inner, 16 / esz);
  if (!flat && vw * esz != 16) return 0;
  const int nb = (n + bl - 1) / bl;
  const int64_t nc = (int64_t)P.pv * nb;
  const int tiles = max_orbit_tiles(P.G, (int)std::min<int64_t>(nc, 64));
  int64_t ts = ipow(bl, d) * inner;
  if (flat) ts = (ts + 16 / esz + 16 / esz - 1) / (16 / esz) * (16 / esz);
  if (vw_out) *vw_out = vw;
  return ((int64_t)tiles * ts * esz + 15) / 16 * 16 + ipow(bl, d) * 4;
}

// Default tile edge: the largest usable bl whose orbit fits 32 KiB of LDS,
// else 64 KiB, else the LDS of a CU (the rules of the group form).
static spinsum_status choose_pair_tile(const spinsum_plan_s& P, spinsum_tile_t* tile) {
  const int64_t budget = P.lds_limit - 512;
  for (int64_t cap : {(int64_t)32 * 1024, (int64_t)64 * 1024, budget}) {
    for (int bl = std::min(P.n, 255); bl >= 1; --bl) {
      const int64_t b = pair_lds_bytes(P, bl, nullptr);
      if (b > 0 && b <= std::min(cap, budget)) {
        spinsum_tile_t t{};
        t.bl = bl;
        t.cubes_per_wg = 1;
        t.variant = SPINSUM_VARIANT_DIRECT_LDS;
        *tile = t;
        return SPINSUM_OK;
      }
    }
  }
  return SPINSUM_ERR_UNSUPPORTED;
}

static spinsum_status build_pair_tiling(spinsum_plan_s* P, const spinsum_tile_t& tile) {
  const int n = P->n, d = P->d, inner = P->inner, esz = elem_size(*P);
  const int64_t V = P->pv;
  Tiling T;
  PairGeom pg;
  std::memset(&pg, 0, sizeof(pg));
  std::vector<uint64_t> orbits;
  const int bl = tile.bl <= 0 ? n : std::min(tile.bl, n);
  if (bl < 1 || bl > 255) return SPINSUM_ERR_UNSUPPORTED;
  int vw = 1;
  const int64_t lds_bytes = pair_lds_bytes(*P, bl, &vw);
  if (lds_bytes == 0) return SPINSUM_ERR_UNSUPPORTED;
  const bool flat = (bl == n);
  const int nb = (n + bl - 1) / bl;
  const int64_t nc = V * nb;
  if (nc > 16000) return SPINSUM_ERR_UNSUPPORTED;  // 16-bit combined blocks
  Geom& g = T.g;
  g.ncubes = P->ncubes;
  g.n = n;
  g.bl = bl;
  g.cpw = 1;
  g.ngroups = 1;
  for (int m = 0; m < kMaxD; ++m) g.gst[m] = 0;
  for (int m = 0; m < d; ++m) g.gst[m] = (int32_t)(ipow(n, d - 1 - m) * inner);
  lds_strides(d, bl, 0, inner, g.lst, &g.ts);
  g.cube_lds = g.ts;
  g.rows = (int32_t)ipow(bl, d - 1);
  g.vpr = flat ? 1 : bl * inner / vw;
  g.inner = inner;
  g.fd_vpr = make_fastdiv((uint32_t)g.vpr);
  g.fd_rows = make_fastdiv((uint32_t)g.rows);
  g.fd_bl = make_fastdiv((uint32_t)bl);
  g.fd_ngroups = make_fastdiv(1);
  g.fd_inner = make_fastdiv((uint32_t)inner);
  const int64_t group_elems = ipow(n, d) * inner;
  int64_t block = group_elems;
  for (int m = 0; m < d; ++m) {
    if (block > ((int64_t)1 << 62) / V) return SPINSUM_ERR_UNSUPPORTED;
    block *= V;
  }
  g.cube_elems = block;
  for (int m = 0; m < d; ++m) pg.pstride[m] = ipow(V, d - 1 - m) * group_elems;
  pg.nc = (int32_t)nc;
  pg.nb = nb;
  pg.last_ext = n - (nb - 1) * bl;
  pg.flat = flat ? 1 : 0;
  pg.tile_stride = flat ? (int32_t)((g.ts + 16 / esz + 16 / esz - 1) / (16 / esz) * (16 / esz)) : g.ts;
  pg.fd_nb = make_fastdiv((uint32_t)nb);
  pg.norb = multiset_count(nc, d);
  // host table of 8 bytes per orbit (plus the sort for the line order)
  if (pg.norb <= 0 || pg.norb > (1ll << 26)) return SPINSUM_ERR_UNSUPPORTED;
  pg.fd_norb = make_fastdiv((uint32_t)pg.norb);
  T.nitems = P->ncubes * pg.norb;
  if (T.nitems >= (1ll << 31) - 8) return SPINSUM_ERR_UNSUPPORTED;
  // the orbit table: sorted combined-block tuples in lexicographic order
  orbits.reserve((size_t)pg.norb);
  {
    std::vector<int> c(d, 0);
    while (true) {
      uint64_t pk = 0;
      for (int m = 0; m < d; ++m) pk |= (uint64_t)c[m] << (16 * m);
      orbits.push_back(pk);
      int m = d - 1;
      while (m >= 0 && c[m] == nc - 1) --m;
      if (m < 0) break;
      c[m]++;
      for (int j = m + 1; j < d; ++j) c[j] = c[m];
    }
  }
  if ((int64_t)orbits.size() != pg.norb) return SPINSUM_ERR_UNSUPPORTED;
  // Orbits whose tiles share cache lines along the fastest axis get
  // neighbouring item numbers (same XCD, close in time): key = the multiset
  // of (a_m, b_m / s) with s blocks per 128-byte line, or every block of the
  // axis when group rows are not whole lines.  Loop-nest order within a key.
  if (!flat && orbits.size() > 128 && orbits.size() <= ((size_t)1 << 24)) {  // sort buffer <= 384 MiB
    const int64_t row = (int64_t)bl * inner * esz;
    const int64_t line = 128;
    int s = nb;
    if (((int64_t)n * inner * esz) % line == 0 && row < line && line % row == 0) s = (int)(line / row);
    if (s > 1) {
      struct Keyed {
        uint32_t k[kMaxD];
        uint64_t v;
      };
      std::vector<Keyed> kv(orbits.size());
      for (size_t i = 0; i < orbits.size(); ++i) {
        Keyed& e = kv[i];
        for (int m = 0; m < kMaxD; ++m) e.k[m] = 0;
        for (int m = 0; m < d; ++m) {
          const int cm = (int)((orbits[i] >> (16 * m)) & 0xFFFFu);
          e.k[m] = ((uint32_t)(cm / nb) << 16) | (uint32_t)((cm % nb) / s);
        }
        std::sort(e.k, e.k + d);
        e.v = orbits[i];
      }
      std::stable_sort(kv.begin(), kv.end(), [](const Keyed& x, const Keyed& y) {
        return std::lexicographical_compare(x.k, x.k + kMaxD, y.k, y.k + kMaxD);
      });
      for (size_t i = 0; i < orbits.size(); ++i) orbits[i] = kv[i].v;
    }
  }
  // representative lists per key (equal-neighbour mask, ragged-block mask)
  for (int key = 0; key < (1 << (2 * d - 1)); ++key) {
    int ext[kMaxD];
    bool consistent = true;
    for (int m = 0; m < d; ++m) ext[m] = ((key >> (d - 1 + m)) & 1) ? pg.last_ext : bl;
    for (int m = 0; m + 1 < d; ++m)
      if (((key >> m) & 1) && ext[m] != ext[m + 1]) consistent = false;
    pg.rep_off[key] = (int32_t)T.reps.size();
    if (consistent) {
      int64_t box = 1;
      for (int m = 0; m < d; ++m) box *= ext[m];
      std::vector<int> l(d, 0);
      for (int64_t e = 0; e < box; ++e) {
        int64_t rem = e;
        for (int m = d - 1; m >= 0; --m) {
          l[m] = (int)(rem % ext[m]);
          rem /= ext[m];
        }
        bool ok = true;
        for (int m = 0; m + 1 < d; ++m)
          if (((key >> m) & 1) && l[m] > l[m + 1]) ok = false;
        if (!ok) continue;
        uint32_t pk = 0;
        for (int m = 0; m < d; ++m) pk |= (uint32_t)l[m] << (8 * m);
        T.reps.push_back(pk);
      }
      if (inner == 1) order_reps_for_banks(T.reps, (size_t)pg.rep_off[key], P->G, g.lst, esz, bl);
    }
    pg.rep_cnt[key] = (int32_t)T.reps.size() - pg.rep_off[key];
    T.max_rep_cnt = std::max(T.max_rep_cnt, pg.rep_cnt[key]);
  }
  T.nb = nb;
  T.vw = vw;
  T.ragged = (pg.last_ext != bl) ? 1 : 0;
  T.max_orbit_tiles = max_orbit_tiles(P->G, (int)std::min<int64_t>(nc, 64));
  T.max_tiles = T.max_orbit_tiles;
  T.lds_elems = (int64_t)T.max_tiles * pg.tile_stride;
  T.chunks_per_thread = (int)(((int64_t)T.max_tiles * g.rows * g.vpr + 255) / 256);
  T.fits = (lds_bytes <= P->lds_limit) ? 1 : 0;
  if (!T.fits && !(P->flags & SPINSUM_FLAG_HOST_ONLY)) return SPINSUM_ERR_UNSUPPORTED;
  P->T = std::move(T);
  P->pg = pg;
  P->pair_orbits = std::move(orbits);
  return SPINSUM_OK;
}

static spinsum_status apply_pair_tile(spinsum_plan_s* P, const spinsum_tile_t* req) {
  spinsum_tile_t t{};
  if (req && req->bl > 0) {
    t = *req;
    if (t.threads < 0) t.threads = 0;
  } else if (P->ncubes > 0 && P->elems > 0) {
    spinsum_status st = choose_pair_tile(*P, &t);
    if (st != SPINSUM_OK) return st;
  } else {
    t.bl = std::max(1, P->n);
  }
  if (t.threads != 0 && t.threads != 256 && t.threads != 512 && t.threads != 1024)
    return SPINSUM_ERR_UNSUPPORTED;
  if (t.variant != SPINSUM_VARIANT_AUTO && t.variant != SPINSUM_VARIANT_DIRECT_LDS)
    return SPINSUM_ERR_UNSUPPORTED;
  if (P->flags & SPINSUM_FLAG_NO_DIRECT_LDS) return SPINSUM_ERR_UNSUPPORTED;
  t.variant = SPINSUM_VARIANT_DIRECT_LDS;
  t.lds_pad = 0;
  t.cubes_per_wg = 1;
  t.item_tiles = 0;
  if (P->ncubes > 0 && P->elems > 0) {
    spinsum_status st = build_pair_tiling(P, t);
    if (st != SPINSUM_OK) return st;
    P->T.nts = choose_nts(*P, P->T, P->pg.norb);
  }
  if (t.threads == 0) {
    // 512 threads wherever two workgroups fit a CU: each item first builds
    // its tile list in one wave, and more waves per item issue its loads
    // sooner afterwards (v=48 o=24, 8^3 tiles: 4.76 against 4.64 TB/s at 256
    // threads, although waves then limit a CU to 4 workgroups instead of 6)
    const int64_t wg = pair_lds_bytes(*P, P->T.g.bl > 0 ? P->T.g.bl : std::max(1, P->n), nullptr);
    const int64_t per_cu = std::max<int64_t>(1, P->lds_limit / std::max<int64_t>(1, wg));
    t.threads = per_cu >= 2 ? 512 : 1024;
  }
  P->tile = t;
  return SPINSUM_OK;
}

static spinsum_status apply_tile(spinsum_plan_s* P, const spinsum_tile_t* req) {
  if (P->pair) return apply_pair_tile(P, req);
  spinsum_tile_t t{};
  bool chosen = false;  // tile picked by the planner (not requested, not cached)
  const int vmax = max_vector_width(*P, (int64_t)std::max(1, P->n) * P->inner);
  if (req && req->bl > 0) {
    t = *req;
    if (t.threads < 0) t.threads = 0;
    if (t.cubes_per_wg <= 0) t.cubes_per_wg = 1;
  } else if (P->n > 0 && P->ncubes > 0) {
    if (!cache_lookup(*P, &t)) {
      spinsum_status st = choose_tile(*P, P->n, P->ncubes, vmax, &t, true);
      if (st != SPINSUM_OK) return st;
      chosen = true;
    }
  }
  if (t.threads != 0 && t.threads != 256 && t.threads != 512 && t.threads != 1024)
    return SPINSUM_ERR_UNSUPPORTED;
  if (t.variant < 0 || t.variant > SPINSUM_VARIANT_LDS_PIPELINE) return SPINSUM_ERR_INVALID_ARG;
  // kernel variant: loads straight into LDS need whole 16-byte rows, except
  // for whole cubes, which the one-shot kernel copies as one contiguous run
  const int bl = t.bl <= 0 ? std::max(1, P->n) : std::min(t.bl, std::max(1, P->n));
  const bool no_direct = (P->flags & SPINSUM_FLAG_NO_DIRECT_LDS) != 0;
  const bool rows_ok =
      vw_for((int64_t)std::max(1, P->n) * P->inner, (int64_t)bl * P->inner, vmax) * elem_size(*P) == 16 &&
      !no_direct;
  const bool direct_ok = rows_ok || (bl >= P->n && !no_direct);
  if (t.variant == SPINSUM_VARIANT_AUTO)
    t.variant = direct_ok ? SPINSUM_VARIANT_DIRECT_LDS : SPINSUM_VARIANT_REG_ONESHOT;
  if (t.variant == SPINSUM_VARIANT_LDS_PIPELINE && !rows_ok)
    t.variant = direct_ok ? SPINSUM_VARIANT_DIRECT_LDS : SPINSUM_VARIANT_REG_ONESHOT;
  if (t.variant == SPINSUM_VARIANT_DIRECT_LDS && !direct_ok) t.variant = SPINSUM_VARIANT_REG_ONESHOT;
  if (t.variant == SPINSUM_VARIANT_DIRECT_LDS || t.variant == SPINSUM_VARIANT_LDS_PIPELINE)
    t.lds_pad = 0;  // dense chunk-order layout
  Tiling T;
  spinsum_status st = build_tiling(*P, P->n, P->ncubes, t, vmax, &T);
  if (st != SPINSUM_OK) return st;
  // A workgroup's LDS is sized for the largest item, so where fewer than
  // four fit a CU, one-orbit items of small orbits leave most of a slot
  // unused: pack consecutive orbits up to the largest one instead
  // (measured on one 80^4 / 112^4 FP64 cube: +9 % / +7 %; -3 % on 54^4).
  if (chosen && t.variant == SPINSUM_VARIANT_DIRECT_LDS && t.item_tiles == 0 && bl < P->n &&
      T.orbits.size() > 1) {
    const int64_t wg_lds = (T.lds_elems * elem_size(*P) + 15) / 16 * 16 + (int64_t)T.max_rep_cnt * 4;
    if (P->lds_limit / std::max<int64_t>(1, wg_lds) < 4) {
      t.item_tiles = T.max_orbit_tiles;
      st = build_tiling(*P, P->n, P->ncubes, t, vmax, &T);
      if (st != SPINSUM_OK) return st;
    }
  }
  if (t.variant == SPINSUM_VARIANT_REG_PIPELINE && T.chunks_per_thread > 16)
    t.variant = SPINSUM_VARIANT_REG_ONESHOT;
  // two tile buffers and every representative table must fit in LDS
  if (t.variant == SPINSUM_VARIANT_LDS_PIPELINE &&
      (((int64_t)T.reps.size() * 4 + 15) / 16 * 16 + 2 * ((T.lds_elems * elem_size(*P) + 15) / 16 * 16) >
       P->lds_limit))
    t.variant = SPINSUM_VARIANT_DIRECT_LDS;
  // workgroup size: the direct-LDS kernels take 256, 512 or 1024 threads;
  // by default enough that the workgroups LDS lets onto a CU hold about 16
  // waves (the combine step of big items then spreads over more waves);
  // the register kernels run 256
  if (t.variant != SPINSUM_VARIANT_DIRECT_LDS && t.variant != SPINSUM_VARIANT_LDS_PIPELINE) {
    t.threads = 256;
  } else if (t.threads == 0) {
    const int64_t tiles = (T.lds_elems * elem_size(*P) + 15) / 16 * 16;
    const int64_t wg_lds = (t.variant == SPINSUM_VARIANT_DIRECT_LDS)
                               ? tiles + (int64_t)T.max_rep_cnt * 4
                               : 2 * tiles + ((int64_t)T.reps.size() * 4 + 15) / 16 * 16;
    const int64_t per_cu = std::max<int64_t>(1, P->lds_limit / std::max<int64_t>(1, wg_lds));
    t.threads = per_cu >= 4 ? 256 : per_cu >= 2 ? 512 : 1024;
  }
  T.nts = choose_nts(*P, T, (int64_t)T.orbits.size());
  T.ntl = choose_ntl(*P, T);
  P->tile = t;
  P->T = std::move(T);
  return SPINSUM_OK;
}

static spinsum_status common_checks(int d, spinsum_dtype dtype, int inplace, unsigned flags) {
  if (d < 2 || d > 4) return SPINSUM_ERR_UNSUPPORTED;
  if ((flags & SPINSUM_FLAG_MULTI_PASS) && (flags & SPINSUM_FLAG_CHAIN_STAGES))
    return SPINSUM_ERR_INVALID_ARG;
  if (dtype != SPINSUM_F64 && dtype != SPINSUM_F32) return SPINSUM_ERR_INVALID_ARG;
  if (inplace != 0 && inplace != 1) return SPINSUM_ERR_INVALID_ARG;
  return SPINSUM_OK;
}

// Group extent N, outer spectator cubes (product of the dims before the
// group) and inner spectator run (product of the dims after it; 1 if none).
// An empty inner run makes the tensor empty (no cubes).
static spinsum_status shape_info(int ndim, const int64_t* extents, int group_first, int d,
                                 int* n, int64_t* ncubes, int* inner) {
  if (ndim < 1 || ndim > 64 || extents == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if (group_first < 0 || group_first + d > ndim) return SPINSUM_ERR_INVALID_ARG;
  for (int k = 0; k < ndim; ++k)
    if (extents[k] < 0) return SPINSUM_ERR_INVALID_ARG;
  for (int m = 1; m < d; ++m)
    if (extents[group_first + m] != extents[group_first]) return SPINSUM_ERR_EXTENT_MISMATCH;
  if (extents[group_first] > 255 * 255) return SPINSUM_ERR_UNSUPPORTED;
  *n = (int)extents[group_first];
  int64_t r = 1;
  for (int k = group_first + d; k < ndim; ++k) {
    if (extents[k] > 0 && r > (1ll << 31) / extents[k]) return SPINSUM_ERR_UNSUPPORTED;
    r *= extents[k];
  }
  int64_t c = 1;
  for (int k = 0; k < group_first; ++k) {
    if (extents[k] > 0 && c > (1ll << 62) / extents[k]) return SPINSUM_ERR_UNSUPPORTED;
    c *= extents[k];
  }
  if (r == 0) {
    r = 1;
    c = 0;
  }
  *ncubes = c;
  *inner = (int)r;
  return SPINSUM_OK;
}

// The group axes that some permutation of the operator moves (a term with
// nonzero coefficient in any stage), as the range [*s0, *e0) when they are
// contiguous.  Returns false when no axis moves or the moved axes are not
// contiguous.
static bool moved_axes(const spinsum_plan_s& P, int* s0, int* e0) {
  int lo = P.d, hi = -1;
  std::vector<bool> moved(P.d, false);
  for (const std::vector<double>& st : P.stage_a)
    for (int r = 0; r < P.G.df; ++r) {
      if (st[r] == 0.0) continue;
      for (int m = 0; m < P.d; ++m)
        if (P.G.p[r][m] != m) moved[m] = true;
    }
  for (int m = 0; m < P.d; ++m)
    if (moved[m]) {
      lo = std::min(lo, m);
      hi = std::max(hi, m);
    }
  if (hi < 0) return false;
  for (int m = lo; m <= hi; ++m)
    if (!moved[m]) return false;
  *s0 = lo;
  *e0 = hi + 1;
  return true;
}

// The subgroup reduction (see spinsum_plan in the header): the plan of the
// moved axes [s0, e0), its terms the operator's own ones restricted to
// those axes (they fix every other axis), stage by stage.
static spinsum_status reduce_to_moved_axes(spinsum_plan_s* P, int s0, int e0) {
  const int d2 = e0 - s0;
  const int K = (int)P->stage_a.size();
  std::vector<int> nt(K, 0), pp;
  std::vector<double> aa;
  for (int k = 0; k < K; ++k)
    for (int r = 0; r < P->G.df; ++r) {
      const double a = P->stage_a[k][r];
      if (a == 0.0) continue;
      for (int m = 0; m < d2; ++m) pp.push_back(P->G.p[r][s0 + m] - s0);
      aa.push_back(a);
      ++nt[k];
    }
  if (pp.empty()) {
    pp.push_back(0);
    aa.push_back(0.0);
  }
  spinsum_plan_t sub = nullptr;
  spinsum_status st = spinsum_plan(&sub, P->ndim, P->extents.data(), P->group_first + s0, d2, K,
                                   nt.data(), pp.data(), aa.data(), (spinsum_dtype)P->dtype,
                                   P->inplace, P->flags | SPINSUM_FLAG_FULL_GROUP);
  if (st != SPINSUM_OK) return st;
  P->sub = sub;
  P->sub_first = P->group_first + s0;
  return SPINSUM_OK;
}

extern "C" spinsum_status spinsum_plan(spinsum_plan_t* plan, int ndim, const int64_t* extents,
                                       int group_first, int d, int nstages, const int* nterms,
                                       const int* perms, const double* alpha,
                                       spinsum_dtype dtype, int inplace, unsigned flags) {
  if (plan == nullptr) return SPINSUM_ERR_INVALID_ARG;
  *plan = nullptr;
  spinsum_status st = common_checks(d, dtype, inplace, flags);
  if (st != SPINSUM_OK) return st;
  int n = 0, inner = 1;
  int64_t ncubes = 0;
  st = shape_info(ndim, extents, group_first, d, &n, &ncubes, &inner);
  if (st != SPINSUM_OK) return st;
  // index-pair form: the d dims before the group are its partners
  bool pair = false;
  int64_t V = 1;
  if (flags & SPINSUM_FLAG_INDEX_PAIRS) {
    if (group_first < d) return SPINSUM_ERR_INVALID_ARG;
    V = extents[group_first - d];
    for (int m = 1; m < d; ++m)
      if (extents[group_first - d + m] != V) return SPINSUM_ERR_EXTENT_MISMATCH;
    if (V > 1 && n == 1) {
      // a group of extent 1: the ordinary summation over the partners
      st = shape_info(ndim, extents, group_first - d, d, &n, &ncubes, &inner);
      if (st != SPINSUM_OK) return st;
    } else if (V > 1 && n > 1) {
      if (V > 16000) return SPINSUM_ERR_UNSUPPORTED;
      pair = true;
      ncubes = 1;
      for (int k = 0; k < group_first - d; ++k) ncubes *= extents[k];
    }
    // V <= 1 or an empty group: the ordinary summation over the group
  }
  spinsum_plan_s* P = new (std::nothrow) spinsum_plan_s();
  if (!P) return SPINSUM_ERR_OUT_OF_MEMORY;
  P->d = d;
  P->n = n;
  P->group_first = group_first;
  P->inner = inner;
  P->pair = pair;
  P->pv = (int)V;
  P->ndim = ndim;
  P->extents.assign(extents, extents + ndim);
  P->ncubes = ncubes;
  P->dtype = dtype;
  P->inplace = inplace;
  P->flags = flags;
  P->G.init(d);
  if (n > 0 && ipow(n, d) * inner >= (1ll << 31)) {
    delete P;
    return SPINSUM_ERR_UNSUPPORTED;
  }
  P->elems = ncubes * ipow(n, d) * inner;
  if (pair) {
    const int64_t vd = ipow(V, d);
    if (P->elems > 0 && vd > ((int64_t)1 << 62) / P->elems) {
      delete P;
      return SPINSUM_ERR_UNSUPPORTED;
    }
    P->elems *= vd;
  }
  st = set_terms(P, nstages, nterms, perms, alpha);
  if (st == SPINSUM_OK) {
    query_device(P);
    st = apply_tile(P, nullptr);
  }
  if (st == SPINSUM_OK) st = upload_tables(P);
  int s0 = 0, e0 = 0;
  if (st == SPINSUM_OK && !(flags & (SPINSUM_FLAG_FULL_GROUP | SPINSUM_FLAG_INDEX_PAIRS)) &&
      !pair && P->elems > 0 && moved_axes(*P, &s0, &e0) && e0 - s0 >= 2 && e0 - s0 < d)
    st = reduce_to_moved_axes(P, s0, e0);
  if (st != SPINSUM_OK) {
    spinsum_plan_destroy(P);
    return st;
  }
  *plan = P;
  return SPINSUM_OK;
}

// Tables of a batched plan for one choice of the whole-cube item size
// (item_bytes 0: the default rule below).  Also used by the autotuner.
spinsum_status spinsum::build_batched(spinsum_plan_s* P, int64_t item_bytes) {
  const int nblocks = P->nblocks, d = P->d;
  const std::vector<int>& ns = P->bns;
  const std::vector<int64_t>& cs = P->bcs;
  const std::vector<int>& rs = P->brs;
  spinsum_status st = SPINSUM_OK;
  P->btil.clear();
  P->blocks.clear();
  P->block_elems.clear();
  P->items.clear();
  P->elems = 0;
  P->ncubes = 0;
  P->batch_lds_elems = 0;
  P->batch_rep_bytes = 0;
  // tiles: whole cubes when they fit (copied as one contiguous run, any
  // extent), packed up to the largest cube of the batch (at least 8 KiB, at
  // most 40 KiB) so that every workgroup moves about the same bytes; tile
  // orbits through registers otherwise, with one vector width for all such
  // blocks
  const int esz = elem_size(*P);
  auto cube_bytes_of = [&](int b) { return ipow(ns[b], d) * rs[b] * esz; };
  int64_t target = 8 * 1024;
  for (int b = 0; b < nblocks; ++b)
    if (ns[b] > 0 && cs[b] > 0 && cube_bytes_of(b) <= 40 * 1024)
      target = std::max<int64_t>(target, cube_bytes_of(b));
  if (item_bytes > 0) target = item_bytes;
  int vmax = 16 / esz;
  for (int b = 0; b < nblocks; ++b)
    if (ns[b] > 0 && cs[b] > 0 && cube_bytes_of(b) > 40 * 1024)
      vmax = std::min(vmax, max_vector_width(*P, (int64_t)ns[b] * rs[b]));
  P->batch_vw = vmax;
  P->btil.resize(nblocks);
  P->blocks.resize(nblocks);
  P->block_elems.resize(nblocks);
  int group_base = 0;
  for (int b = 0; b < nblocks; ++b) {
    spinsum_tile_t t{};
    // the tile rules read the inner spectator run from the plan: set it to
    // this block's for the block's tables (reset to 1 below)
    P->inner = rs[b];
    if (ns[b] > 0 && cs[b] > 0) {
      const int64_t cube_bytes = cube_bytes_of(b);
      if (cube_bytes <= 40 * 1024) {
        t.bl = ns[b];
        t.cubes_per_wg = (int)std::max<int64_t>(1, std::min<int64_t>(target / cube_bytes, cs[b]));
        t.threads = 256;
        t.lds_pad = 0;
      } else {
        st = choose_tile(*P, ns[b], cs[b], vmax, &t, false);
        if (st == SPINSUM_OK && t.bl >= ns[b]) {
          // a whole cube after all (up to 64 KiB): the batched kernel copies
          // whole cubes as one contiguous run, so their LDS image is unpadded
          t.bl = ns[b];
          t.cubes_per_wg = 1;
          t.lds_pad = 0;
          t.threads = 256;
        }
        if (st == SPINSUM_OK && ((int64_t)t.bl * rs[b]) % vmax != 0 && t.bl != ns[b])
          st = SPINSUM_ERR_UNSUPPORTED;
      }
    }
    if (st == SPINSUM_OK) st = build_tiling(*P, ns[b], cs[b], t, vmax, &P->btil[b]);
    P->inner = 1;
    if (st != SPINSUM_OK) return st;
    Tiling& T = P->btil[b];
    std::memset(&P->blocks[b], 0, sizeof(BatchBlock));
    P->blocks[b].g = T.g;
    P->blocks[b].group_base = group_base;
    P->block_elems[b] = (ns[b] > 0 ? cs[b] * ipow(ns[b], d) * rs[b] : 0);
    P->elems += P->block_elems[b];
    P->ncubes += cs[b];
    P->batch_lds_elems = std::max(P->batch_lds_elems, T.lds_elems);
    P->batch_rep_bytes = std::max<int64_t>(P->batch_rep_bytes, (int64_t)T.max_rep_cnt * 4);
    // items of this block
    const Geom& g = T.g;
    if (T.nitems > 0) {
      if (g.bl == g.n) {
        for (int64_t c0 = 0; c0 < g.ncubes; c0 += g.cpw) {
          BatchItem it{};
          it.cube0 = c0;
          it.block = b;
          it.group = group_base;
          it.ncubes = (int32_t)std::min<int64_t>(g.cpw, g.ncubes - c0);
          P->items.push_back(it);
        }
      } else {
        for (int64_t c = 0; c < g.ncubes; ++c)
          for (int o = 0; o < g.ngroups; ++o) {
            BatchItem it{};
            it.cube0 = c;
            it.block = b;
            it.group = group_base + o;
            it.ncubes = 1;
            P->items.push_back(it);
          }
      }
    }
    group_base += (int)T.groups.size();
  }
  // larger items first: the workgroups dispatched last then get the small ones
  auto cost = [&](const BatchItem& it) {
    const Tiling& T = P->btil[it.block];
    const GroupDev& gd = T.groups[it.group - P->blocks[it.block].group_base];
    int64_t tile = ipow(T.g.bl, d) * T.g.inner;
    return (int64_t)it.ncubes * gd.ntiles * tile;
  };
  std::stable_sort(P->items.begin(), P->items.end(),
                   [&](const BatchItem& a, const BatchItem& b) { return cost(a) > cost(b); });
  if ((int64_t)P->items.size() >= (1ll << 31)) return SPINSUM_ERR_UNSUPPORTED;
  // behind the tiles: the representative lists (whole cubes) or the tile
  // table (tile orbits)
  P->batch_rep_bytes = std::max<int64_t>(P->batch_rep_bytes, 2 * kMaxDF * 4);
  if ((P->batch_lds_elems * elem_size(*P) + 15) / 16 * 16 + P->batch_rep_bytes > P->lds_limit)
    return SPINSUM_ERR_UNSUPPORTED;
  P->batch_grid = (int)std::min<int64_t>((int64_t)P->items.size(), INT32_MAX);
  P->batch_item_bytes = target;
  return SPINSUM_OK;
}

extern "C" spinsum_status spinsum_plan_batched(spinsum_plan_t* plan, int nblocks, const int* ndims,
                                               const int64_t* const* extents, int group_first,
                                               int d, int nstages, const int* nterms,
                                               const int* perms, const double* alpha,
                                               spinsum_dtype dtype, int inplace, unsigned flags) {
  if (plan == nullptr) return SPINSUM_ERR_INVALID_ARG;
  *plan = nullptr;
  spinsum_status st = common_checks(d, dtype, inplace, flags);
  if (st != SPINSUM_OK) return st;
  if (nblocks < 1 || nblocks > (1 << 20) || ndims == nullptr || extents == nullptr)
    return SPINSUM_ERR_INVALID_ARG;
  if (group_first < -1) return SPINSUM_ERR_INVALID_ARG;
  if (flags & SPINSUM_FLAG_INDEX_PAIRS) return SPINSUM_ERR_UNSUPPORTED;
  std::vector<int> ns(nblocks), rs(nblocks);
  std::vector<int64_t> cs(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    if (ndims[b] < d) return SPINSUM_ERR_INVALID_ARG;
    const int gf = group_first < 0 ? ndims[b] - d : group_first;
    st = shape_info(ndims[b], extents[b], gf, d, &ns[b], &cs[b], &rs[b]);
    if (st != SPINSUM_OK) return st;
    if (ns[b] > 0 && ipow(ns[b], d) * rs[b] >= (1ll << 31)) return SPINSUM_ERR_UNSUPPORTED;
  }
  spinsum_plan_s* P = new (std::nothrow) spinsum_plan_s();
  if (!P) return SPINSUM_ERR_OUT_OF_MEMORY;
  P->batched = true;
  P->nblocks = nblocks;
  P->d = d;
  P->dtype = dtype;
  P->inplace = inplace;
  P->flags = flags;
  P->G.init(d);
  st = set_terms(P, nstages, nterms, perms, alpha);
  if (st != SPINSUM_OK) {
    delete P;
    return st;
  }
  query_device(P);
  P->bns = ns;
  P->bcs = cs;
  P->brs = rs;
  {
    int64_t item_bytes = 0;
    int persistent = 0;
    if (batched_cache_lookup(*P, &item_bytes, &persistent)) P->batch_persistent = persistent;
    st = build_batched(P, item_bytes);
  }
  if (st != SPINSUM_OK) {
    delete P;
    return st;
  }
  st = upload_tables(P);
  if (st != SPINSUM_OK) {
    free_device(P);
    delete P;
    return st;
  }
  *plan = P;
  return SPINSUM_OK;
}

extern "C" spinsum_status spinsum_plan_set_tile(spinsum_plan_t P, const spinsum_tile_t* tile) {
  if (P == nullptr || tile == nullptr || P->batched) return SPINSUM_ERR_INVALID_ARG;
  if (P->sub) return spinsum_plan_set_tile(P->sub, tile);
  if (tile->bl < 0 || tile->cubes_per_wg < 0) return SPINSUM_ERR_INVALID_ARG;
  spinsum_tile_t keep = P->tile;
  Tiling keepT = P->T;
  const PairGeom keep_pg = P->pg;
  const std::vector<uint64_t> keep_orbits = P->pair_orbits;
  spinsum_status st = apply_tile(P, tile);
  if (st == SPINSUM_OK) st = upload_tables(P);
  if (st != SPINSUM_OK) {
    P->tile = keep;
    P->T = keepT;
    P->pg = keep_pg;
    P->pair_orbits = keep_orbits;
    spinsum_status st2 = upload_tables(P);
    (void)st2;
  }
  return st;
}

extern "C" spinsum_status spinsum_plan_get_info(spinsum_plan_t P, spinsum_plan_info_t* info) {
  if (P == nullptr || info == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if (P->sub) {
    // the tiling of the group the kernels permute; the operator's own size
    spinsum_status st = spinsum_plan_get_info(P->sub, info);
    if (st != SPINSUM_OK) return st;
    info->d = P->d;
    info->elems = P->elems;
    int nz = 0;
    for (double v : P->expanded) nz += (v != 0.0);
    info->nterms_expanded = nz;
    info->exec_group_first = P->sub_first;
    info->coef_grad_split = P->cg_split ? 1 : 0;  // the gradient runs on the whole group
    info->unpack_bl = P->pk_own ? P->Tu.g.bl : P->T.g.bl;  // and so does unpacking
    info->unpack_persistent =
        (P->pk_own && P->pk_persist && !(P->flags & SPINSUM_FLAG_NO_XCD_REMAP)) ? 1 : 0;
    info->unpack_nt_stores = (P->pk_own ? P->Tu.nts : P->T.nts) != 0 ? 1 : 0;
    return SPINSUM_OK;
  }
  std::memset(info, 0, sizeof(*info));
  info->exec_d = P->d;
  info->exec_group_first = P->group_first;
  const int v = P->tile.variant;
  // (the register pipeline runs one-shot where the plan picked cached stores)
  if ((P->batched && P->batch_persistent) ||
      (!P->batched && !P->pair &&
       ((v == SPINSUM_VARIANT_REG_PIPELINE && P->T.nts) || v == SPINSUM_VARIANT_LDS_PIPELINE)))
    info->persistent_per_cu = P->occ_blocks;
  info->d = P->d;
  info->n = P->n;
  info->ncubes = P->ncubes;
  info->elems = P->elems;
  info->nstages = (int)P->stage_a.size();
  int nz = 0;
  for (double v : P->expanded) nz += (v != 0.0);
  info->nterms_expanded = nz;
  info->nblocks = P->nblocks;
  info->dtype = P->dtype;
  info->inplace = P->inplace;
  info->threads = P->batched ? 256 : P->tile.threads;
  info->inner = P->inner;
  info->pair_extent = P->pair ? P->pv : 0;
  info->nt_stores = P->batched ? 1 : P->T.nts;
  info->nt_loads = P->batched ? 1 : P->T.ntl;
  info->coef_grad_split = P->cg_split ? 1 : 0;
  info->unpack_bl = (P->batched || P->pair) ? 0 : P->pk_own ? P->Tu.g.bl : P->T.g.bl;
  info->unpack_nt_stores =
      (!P->batched && !P->pair && (P->pk_own ? P->Tu.nts : P->T.nts) != 0) ? 1 : 0;
  info->unpack_persistent = (!P->batched && !P->pair && P->pk_own && P->pk_persist &&
                        !(P->flags & SPINSUM_FLAG_NO_XCD_REMAP)) ? 1 : 0;
  info->batch_item_bytes = P->batched ? P->batch_item_bytes : 0;
  info->batch_persistent = P->batched ? P->batch_persistent : 0;
  if (!P->batched) {
    info->bl = P->T.g.bl;
    info->variant = P->tile.variant;
    info->lds_pad = P->tile.lds_pad;
    info->nb = P->T.nb;
    info->norbits = (int)P->T.orbits.size();
    info->items_per_cube = P->T.g.ngroups;
    info->item_tiles = P->T.max_tiles;
    info->cubes_per_wg = P->T.g.cpw;
    info->max_tiles = P->T.max_tiles;
    info->lds_bytes = P->T.lds_elems * elem_size(*P);
    info->nitems = P->T.nitems;
    info->vector_width = P->T.vw;
    info->ragged = P->T.ragged;
    info->fits_lds = P->T.fits;
    info->rep_lds_bytes = (int64_t)P->T.max_rep_cnt * 4;
    info->chunks_per_thread = P->T.chunks_per_thread;
    if (P->pair) {
      info->norbits = (int)std::min<int64_t>(P->pg.norb, INT32_MAX);
      info->items_per_cube = info->norbits;
    }
  } else {
    info->lds_bytes = P->batch_lds_elems * elem_size(*P);
    info->nitems = (int64_t)P->items.size();
    info->vector_width = P->batch_vw;
    int norb = 0, mt = 0;
    for (const Tiling& t : P->btil) {
      norb += (int)t.orbits.size();
      mt = std::max(mt, t.max_tiles);
      info->ragged |= t.ragged;
    }
    info->norbits = norb;
    info->max_tiles = mt;
    info->fits_lds = (P->batch_lds_elems * elem_size(*P) + 15) / 16 * 16 + P->batch_rep_bytes <= P->lds_limit;
  }
  return SPINSUM_OK;
}

extern "C" spinsum_status spinsum_plan_expanded(spinsum_plan_t P, int cap, int* nterms, int* perms,
                                                double* alpha) {
  if (P == nullptr || nterms == nullptr || cap < 0) return SPINSUM_ERR_INVALID_ARG;
  int k = 0;
  for (int r = 0; r < P->G.df; ++r) {
    if (P->expanded[r] == 0.0) continue;
    if (k < cap) {
      if (perms == nullptr || alpha == nullptr) return SPINSUM_ERR_INVALID_ARG;
      for (int m = 0; m < P->d; ++m) perms[k * P->d + m] = P->G.p[r][m];
      alpha[k] = P->expanded[r];
    }
    ++k;
  }
  *nterms = k;
  return SPINSUM_OK;
}

// Replays, on the host, the addresses one work item computes on the device
// (load, combine, store) with the kernels' own index functions, and checks
// that they stay in bounds and agree with each other.
// Combine step of a work item: for every orbit of the group, the LDS
// address of sigma . x (plus the item's LDS shift) holds global element
// sigma . x.
template <int D>
static bool check_combine(const Tiling& T, const GroupDev& gd, int ncub,
                          const std::vector<int64_t>& lds_of, int shift, std::string* why) {
  const Geom& g = T.g;
  const int d = D;
  for (int k = 0; k < gd.norb; ++k) {
    const uint32_t nrep = (uint32_t)ncub * (uint32_t)gd.rep_cnt[k];
    int x0[D];  // origin of the orbit's identity tile
    {
      int64_t o0 = gd.tile_off[gd.slot_base[k][0] / g.ts];
      for (int m = 0; m < d; ++m) x0[m] = (int)((o0 / g.gst[m]) % g.n);
    }
    for (uint32_t i = 0; i < nrep * (uint32_t)g.inner; ++i) {
      // unit -> (cube, representative, inner index), inner index fastest
      const uint32_t j = fdiv(i, g.fd_inner);
      const uint32_t si = i - j * (uint32_t)g.inner;
      uint32_t ci = (ncub == 1) ? 0u : fdiv(j, gd.fd_rep[k]);
      uint32_t ri = j - ci * (uint32_t)gd.rep_cnt[k];
      if (ci >= (uint32_t)ncub || ri >= (uint32_t)gd.rep_cnt[k]) { *why = "bad representative index"; return false; }
      uint32_t pk = T.reps[gd.rep_off[k] + ri];
      int l[D];
      for (int m = 0; m < d; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
      int x[D];
      for (int m = 0; m < d; ++m) x[m] = x0[m] + l[m];
      int addrs[kMaxDF];
      orbit_addrs<D>(g, (int)ci * g.cube_lds + (int)si, gd.slot_base[k], l, addrs,
                     std::make_integer_sequence<int, Fact<D>()>{});
      for (int r = 0; r < Fact<D>(); ++r) {
        int a = addrs[r] + shift;
        if (a < 0 || a >= T.lds_elems) { *why = "combine address out of bounds"; return false; }
        int64_t want = (int64_t)ci * g.cube_elems + si;
        for (int m = 0; m < d; ++m) want += (int64_t)x[lex_perm(D, r, m)] * g.gst[m];
        if (lds_of[a] != want) { *why = "combine address does not hold sigma . x"; return false; }
      }
    }
  }
  return true;
}

template <int D, int VW>
static bool emulate_item(const Tiling& T, const GroupDev& gd, int ncub, std::string* why) {
  const Geom& g = T.g;
  const int d = D;
  const int64_t span = (int64_t)ncub * g.cube_elems;
  const uint32_t nchunks = (uint32_t)ncub * (uint32_t)gd.ntiles * (uint32_t)g.rows * (uint32_t)g.vpr;
  if ((int64_t)nchunks > (int64_t)T.chunks_per_thread * 256) {
    *why = "item has more chunks than the prefetch buffer holds";
    return false;
  }
  std::vector<int64_t> lds_of(T.lds_elems, -1);  // LDS slot -> element loaded there
  std::vector<int> loaded((size_t)span, 0);
  for (uint32_t c = 0; c < nchunks; ++c) {
    int go = 0;
    int lo = 0;
    if (!chunk_addr<D, VW>(g, c, gd.ntiles, gd.tile_off, gd.tile_ext, gd.ragged != 0, &go, &lo))
      continue;
    if (go < 0 || go + VW > span || (go % VW) != 0) { *why = "global chunk out of bounds"; return false; }
    if (lo < 0 || lo + VW > T.lds_elems) { *why = "LDS chunk out of bounds"; return false; }
    for (int k = 0; k < VW; ++k) {
      if (lds_of[lo + k] != -1) { *why = "LDS slot written twice"; return false; }
      lds_of[lo + k] = go + k;
      loaded[go + k] += 1;
    }
  }
  // every element of the item's tiles is loaded exactly once
  for (int ci = 0; ci < ncub; ++ci)
    for (int s = 0; s < gd.ntiles; ++s) {
      int ext[kMaxD];
      for (int m = 0; m < d; ++m) ext[m] = (gd.tile_ext[s] >> (8 * m)) & 255;
      int64_t cnt = 1;
      for (int m = 0; m < d; ++m) cnt *= ext[m];
      for (int64_t e = 0; e < cnt; ++e) {
        int64_t rem = e, off = (int64_t)ci * g.cube_elems + gd.tile_off[s];
        for (int m = d - 1; m >= 0; --m) {
          off += (rem % ext[m]) * g.gst[m];
          rem /= ext[m];
        }
        for (int si = 0; si < g.inner; ++si)
          if (loaded[off + si] != 1) { *why = "tile element not loaded exactly once"; return false; }
      }
    }
  return check_combine<D>(T, gd, ncub, lds_of, 0, why);
}

// Whole-cube item copied as one contiguous run (direct-LDS kernel): element
// e of the run sits at LDS element shift + e, for every alignment shift the
// copy can take.
template <int D>
static bool emulate_flat(const Tiling& T, const GroupDev& gd, int ncub, int esz, std::string* why) {
  const int64_t span = (int64_t)ncub * T.g.cube_elems;
  for (int shift = 0; shift < 16 / esz; ++shift) {
    if (shift + span > T.lds_elems) { *why = "contiguous copy exceeds the LDS tile area"; return false; }
    std::vector<int64_t> lds_of(T.lds_elems, -1);
    for (int64_t e = 0; e < span; ++e) lds_of[shift + e] = e;
    if (!check_combine<D>(T, gd, ncub, lds_of, shift, why)) return false;
  }
  return true;
}

template <int D>
static bool emulate_all(const Tiling& T, std::string* why, bool flat, int esz) {
  const Geom& g = T.g;
  std::vector<int> ncubs;
  if (g.bl == g.n) {
    ncubs.push_back((int)std::min<int64_t>(g.cpw, g.ncubes));
    if (g.ncubes % g.cpw) ncubs.push_back((int)(g.ncubes % g.cpw));
  } else {
    ncubs.push_back(1);
  }
  for (const GroupDev& gd : T.groups)
    for (int nc : ncubs) {
      bool ok = false;
      if (flat && !emulate_flat<D>(T, gd, nc, esz, why)) return false;
      if (T.vw == 4) ok = emulate_item<D, 4>(T, gd, nc, why);
      else if (T.vw == 2) ok = emulate_item<D, 2>(T, gd, nc, why);
      else ok = emulate_item<D, 1>(T, gd, nc, why);
      if (!ok) return false;
    }
  return true;
}

// Index-pair form: replays every work item of one pair block -- the tile
// list in first-sigma order, the loads (contiguous copies of whole cubes at
// varied alignment shifts, else the 16-byte row chunks of chunk_addr), the
// combine addresses -- and checks that the LDS slot read for sigma holds
// element sigma . x and that every element of the block belongs to exactly
// one element orbit.
template <int D, int VW>
static bool check_pair(const spinsum_plan_s& P, std::string* why) {
  constexpr int DF = Fact<D>();
  const Tiling& T = P.T;
  const Geom& g = T.g;
  const PairGeom& pg = P.pg;
  const int64_t blk = g.cube_elems;
  if (blk > (1 << 24)) { *why = "pair block too large for the checker"; return false; }
  const int64_t tile_elems = (int64_t)g.rows * g.bl * g.inner;
  std::vector<int64_t> owner((size_t)blk, -1);
  int64_t next_id = 0;
  for (int64_t o = 0; o < pg.norb; ++o) {
    int c[D];
    for (int m = 0; m < D; ++m) c[m] = (int)((P.pair_orbits[o] >> (16 * m)) & 0xFFFFu);
    for (int m = 0; m + 1 < D; ++m)
      if (c[m] > c[m + 1] || c[D - 1] >= pg.nc) { *why = "orbit table not sorted"; return false; }
    int slot[DF], nt = 0;
    int64_t toff[DF];
    int32_t text[DF];
    uint64_t keys[DF];
    for (int r = 0; r < DF; ++r) {
      int t[D];
      uint64_t key = 0;
      for (int m = 0; m < D; ++m) {
        t[m] = c[lex_perm(D, r, m)];
        key |= (uint64_t)t[m] << (16 * m);
      }
      int s = -1;
      for (int j = 0; j < nt; ++j)
        if (keys[j] == key) s = j;
      if (s < 0) {
        pair_tile(g, pg, D, t, &toff[nt], &text[nt]);
        keys[nt] = key;
        s = nt++;
      }
      slot[r] = s;
    }
    if (nt > T.max_tiles) { *why = "orbit has more tiles than planned"; return false; }
    std::vector<int64_t> lds_of((size_t)T.lds_elems, -1);
    int shift[DF];
    for (int t = 0; t < nt; ++t) {
      const int64_t base = (int64_t)t * pg.tile_stride;
      shift[t] = pg.flat ? (int)((t + o) % VW) : 0;
      if (pg.flat) {
        if (shift[t] + tile_elems > pg.tile_stride) { *why = "tile copy exceeds its slot"; return false; }
        if (toff[t] < 0 || toff[t] + tile_elems > blk) { *why = "tile outside the pair block"; return false; }
        for (int64_t e = 0; e < tile_elems; ++e) lds_of[base + shift[t] + e] = toff[t] + e;
        continue;
      }
      const int32_t zero = 0;
      int64_t loaded = 0;
      for (uint32_t ch = 0; ch < (uint32_t)(g.rows * g.vpr); ++ch) {
        int go = 0, lo = 0;
        if (!chunk_addr<D, VW>(g, ch, 1, &zero, &text[t], true, &go, &lo)) continue;
        if (lo != (int)ch * VW) { *why = "LDS chunk not in chunk order"; return false; }
        if (toff[t] + go < 0 || toff[t] + go + VW > blk) { *why = "global chunk out of bounds"; return false; }
        for (int k = 0; k < VW; ++k) {
          if (lds_of[base + lo + k] != -1) { *why = "LDS slot written twice"; return false; }
          lds_of[base + lo + k] = toff[t] + go + k;
        }
        loaded += VW;
      }
      int64_t want = g.inner;
      for (int m = 0; m < D; ++m) want *= (text[t] >> (8 * m)) & 255;
      if (loaded != want) { *why = "tile not loaded exactly once"; return false; }
    }
    const int key = pair_key(g, pg, D, c);
    const int cnt = pg.rep_cnt[key];
    if (cnt <= 0) { *why = "empty representative list"; return false; }
    int32_t sb[DF];
    for (int r = 0; r < DF; ++r) sb[r] = slot[r] * pg.tile_stride + shift[slot[r]];
    for (int i = 0; i < cnt; ++i) {
      const uint32_t pk = T.reps[pg.rep_off[key] + i];
      int l[D];
      for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
      for (int si = 0; si < g.inner; ++si) {
        int addrs[DF];
        orbit_addrs<D>(g, si, sb, l, addrs, std::make_integer_sequence<int, DF>{});
        const int64_t id = next_id++;
        for (int r = 0; r < DF; ++r) {
          const int a = addrs[r];
          if (a < 0 || a >= T.lds_elems) { *why = "combine address out of bounds"; return false; }
          int64_t want = toff[slot[r]] + si;
          for (int m = 0; m < D; ++m) want += (int64_t)l[lex_perm(D, r, m)] * g.gst[m];
          if (lds_of[a] != want) { *why = "combine address does not hold sigma . x"; return false; }
          if (owner[want] != -1 && owner[want] != id) { *why = "element owned twice"; return false; }
          owner[want] = id;
        }
      }
    }
  }
  for (int64_t e = 0; e < blk; ++e)
    if (owner[e] == -1) { *why = "element not owned"; return false; }
  return true;
}

extern "C" spinsum_status spinsum_plan_check_ownership(spinsum_plan_t P, int block, const char** why) {
  static thread_local std::string msg;
  auto fail = [&](const std::string& m) {
    msg = m;
    if (why) *why = msg.c_str();
    return SPINSUM_ERR_INVALID_ARG;
  };
  if (why) *why = "";
  if (P == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if (P->sub) return spinsum_plan_check_ownership(P->sub, block, why);
  if (block < 0 || block >= P->nblocks) return SPINSUM_ERR_INVALID_ARG;
  const Tiling& T = P->batched ? P->btil[block] : P->T;
  const Geom& g = T.g;
  if (g.n <= 0 || g.ncubes <= 0) return SPINSUM_OK;
  if (P->pair) {
    std::string w;
    const int vw = 16 / elem_size(*P);
    bool ok;
    if (P->d == 2) ok = (vw == 2) ? check_pair<2, 2>(*P, &w) : check_pair<2, 4>(*P, &w);
    else if (P->d == 3) ok = (vw == 2) ? check_pair<3, 2>(*P, &w) : check_pair<3, 4>(*P, &w);
    else ok = (vw == 2) ? check_pair<4, 2>(*P, &w) : check_pair<4, 4>(*P, &w);
    if (!ok) return fail(w);
    return SPINSUM_OK;
  }
  const int d = P->d, df = P->G.df, n = g.n, bl = g.bl;
  // every orbit of the cube belongs to exactly one work item
  std::vector<int> orbit_in(T.orbits.size(), 0);
  std::vector<int64_t> owner((size_t)g.cube_elems, -1);
  int64_t next_id = 0;  // one per element orbit (representative, inner index)
  for (const GroupDev& gd : T.groups) {
    int tiles = 0;
    for (int k = 0; k < gd.norb; ++k) {
      // identify the orbit by its identity tile
      int s0 = gd.slot_base[k][0] / g.ts;
      int B[kMaxD];
      for (int m = 0; m < d; ++m) B[m] = (gd.tile_off[s0] / g.gst[m]) % n / bl;
      int match = -1;
      for (size_t o = 0; o < T.orbits.size(); ++o) {
        bool same = true;
        for (int m = 0; m < d; ++m) same = same && T.orbits[o].B[m] == B[m];
        if (same) match = (int)o;
      }
      if (match < 0) return fail("work item holds an unknown orbit");
      orbit_in[match] += 1;
      const OrbitHost& oh = T.orbits[match];
      tiles += oh.ntiles;
      for (int r = 0; r < df; ++r) {
        // the tile recorded for sigma must be sigma . B
        int s = gd.slot_base[k][r] / g.ts;
        if (s < 0 || s >= gd.ntiles || gd.slot_base[k][r] != s * g.ts) return fail("bad slot");
        int64_t off = 0;
        for (int m = 0; m < d; ++m) off += (int64_t)B[P->G.p[r][m]] * bl * g.gst[m];
        if (off != gd.tile_off[s]) return fail("slot table does not match sigma . B");
      }
      for (int i = 0; i < gd.rep_cnt[k]; ++i) {
        uint32_t pk = T.reps[gd.rep_off[k] + i];
        int x[kMaxD];
        for (int m = 0; m < d; ++m) {
          int l = (pk >> (8 * m)) & 255;
          if (l >= std::min(bl, n - B[m] * bl)) return fail("representative outside its tile");
          x[m] = B[m] * bl + l;
        }
        for (int si = 0; si < g.inner; ++si) {
          const int64_t id = next_id++;
          for (int r = 0; r < df; ++r) {
            int64_t e = si;
            for (int m = 0; m < d; ++m) e += (int64_t)x[P->G.p[r][m]] * g.gst[m];
            if (owner[e] != -1 && owner[e] != id) return fail("element owned twice");
            owner[e] = id;
          }
        }
      }
    }
    if (tiles != gd.ntiles) return fail("work item tile count");
  }
  for (int c : orbit_in)
    if (c != 1) return fail("tile orbit not in exactly one work item");
  for (int64_t e = 0; e < g.cube_elems; ++e)
    if (owner[e] == -1) return fail("element not owned");
  std::string w;
  // whole cubes are also copied as one contiguous run by the direct-LDS
  // kernels (single tensors) and by the batched kernel
  const bool flat = (g.bl == g.n) &&
                    (P->batched || P->tile.variant == SPINSUM_VARIANT_DIRECT_LDS);
  const int esz = elem_size(*P);
  bool ok = (d == 2)   ? emulate_all<2>(T, &w, flat, esz)
            : (d == 3) ? emulate_all<3>(T, &w, flat, esz)
                       : emulate_all<4>(T, &w, flat, esz);
  if (!ok) return fail(w);
  return SPINSUM_OK;
}

extern "C" void spinsum_plan_destroy(spinsum_plan_t P) {
  if (!P) return;
  if (P->sub) spinsum_plan_destroy(P->sub);
  free_device(P);
  delete P;
}

extern "C" int spinsum_plan_last_hip_error(spinsum_plan_t P) {
  if (!P) return 0;
  if (P->last_hip_error == 0 && P->sub) return P->sub->last_hip_error;
  return P->last_hip_error;
}

extern "C" const char* spinsum_status_string(spinsum_status s) {
  switch (s) {
    case SPINSUM_OK: return "ok";
    case SPINSUM_ERR_INVALID_ARG: return "invalid argument";
    case SPINSUM_ERR_NOT_PERMUTATION: return "a term is not a permutation";
    case SPINSUM_ERR_EXTENT_MISMATCH: return "group extents differ";
    case SPINSUM_ERR_UNSUPPORTED: return "unsupported configuration";
    case SPINSUM_ERR_ALIASING: return "out-of-place buffers overlap";
    case SPINSUM_ERR_MISALIGNED: return "tensor pointer not 16-byte aligned";
    case SPINSUM_ERR_OUT_OF_MEMORY: return "out of memory";
    case SPINSUM_ERR_HIP: return "HIP runtime error";
    case SPINSUM_ERR_NO_DEVICE: return "plan has no device tables";
  }
  return "unknown status";
}

extern "C" const char* spinsum_version(void) { return "spinsum 0.1 (gfx950)"; }
