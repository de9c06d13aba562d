// spinsum_tune.cpp -- tile autotuner of libspinsum and its cache file.
//
// The tile edge bl of the blocked schedule trades contiguous bytes per row
// (bl * sizeof(T) along the stride-one axis) against LDS per workgroup
// (the largest tile orbit), i.e. against how many workgroups a CU can keep
// in flight.  The paper picks bl from the cache size (Sec. 4.5, Eq. 11);
// here the candidates are timed on the device and the winner is kept.
//
// Cache file: plain text, one line per configuration:
//   <key> <bl> <cubes_per_wg> <threads> <lds_pad> <variant> <item_tiles> <ms>
// key = d<d>_n<N>_r<inner run>_<f64|f32>_ip<0|1>_c<floor(log2(ncubes))>_<arch>.
// Batched plans: <key> <whole-cube item KiB> <persistent 0|1> <ms>, with
// key = batch_b<blocks>_e<elements>_d<d>_<f64|f32>_ip<0|1>_<arch>.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "spinsum_plan_host.h"

namespace spinsum {

static std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (device < 0 || hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return "gfx950";
  }
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  if (c != std::string::npos) a = a.substr(0, c);
  return a.empty() ? std::string("gfx950") : a;
}

static std::string cache_key(const spinsum_plan_s& P) {
  int lg = 0;
  while ((1ll << (lg + 1)) <= P.ncubes) ++lg;
  std::ostringstream os;
  os << "d" << P.d << "_n" << P.n << "_r" << P.inner << "_"
     << (P.dtype == SPINSUM_F32 ? "f32" : "f64") << "_ip" << P.inplace << "_c" << lg << "_"
     << arch_name(P.device);
  return os.str();
}

static std::string batched_key(const spinsum_plan_s& P) {
  int64_t elems = 0;
  for (size_t b = 0; b < P.bns.size(); ++b) {
    int64_t c = P.bcs[b] * (b < P.brs.size() ? P.brs[b] : 1);
    for (int m = 0; m < P.d; ++m) c *= P.bns[b];
    elems += c;
  }
  std::ostringstream os;
  os << "batch_b" << P.nblocks << "_e" << elems << "_d" << P.d << "_"
     << (P.dtype == SPINSUM_F32 ? "f32" : "f64") << "_ip" << P.inplace << "_" << arch_name(P.device);
  return os.str();
}

bool batched_cache_lookup(const spinsum_plan_s& P, int64_t* item_bytes, int* persistent) {
  const char* path = std::getenv("SPINSUM_AUTOTUNE_CACHE");
  if (path == nullptr || *path == 0) return false;
  std::ifstream f(path);
  if (!f) return false;
  const std::string key = batched_key(P);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    int64_t kib = 0;
    int pers = 0;
    double ms = 0;
    if (!(is >> k >> kib >> pers >> ms) || k != key) continue;
    if (kib < 1 || kib > 160 || (pers != 0 && pers != 1)) continue;
    *item_bytes = kib * 1024;
    *persistent = pers;
    found = true;  // the last matching line wins
  }
  return found;
}

static void write_cache_line(const char* path, const std::string& key, const std::string& line) {
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string l;
    while (f && std::getline(f, l)) {
      std::istringstream is(l);
      std::string k;
      if (is >> k && k == key) continue;
      if (!l.empty()) keep.push_back(l);
    }
  }
  keep.push_back(line);
  std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    for (const std::string& l : keep) o << l << "\n";
  }
  std::rename(tmp.c_str(), path);
}

bool cache_lookup(const spinsum_plan_s& P, spinsum_tile_t* tile) {
  const char* path = std::getenv("SPINSUM_AUTOTUNE_CACHE");
  if (path == nullptr || *path == 0) return false;
  std::ifstream f(path);
  if (!f) return false;
  const std::string key = cache_key(P);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    spinsum_tile_t t{};
    double ms = 0;
    if (!(is >> k >> t.bl >> t.cubes_per_wg >> t.threads >> t.lds_pad >> t.variant >> t.item_tiles >> ms))
      continue;
    if (k != key) continue;
    if (t.bl < 1 || t.bl > P.n || t.cubes_per_wg < 1) continue;
    if (t.variant < 0 || t.variant > SPINSUM_VARIANT_LDS_PIPELINE) continue;
    *tile = t;  // the last matching line wins
    found = true;
  }
  return found;
}

static void cache_store(const spinsum_plan_s& P, const char* path, const spinsum_tile_t& t,
                        float ms) {
  const std::string key = cache_key(P);
  std::ostringstream os;
  os << key << " " << t.bl << " " << t.cubes_per_wg << " " << t.threads << " " << t.lds_pad << " "
     << t.variant << " " << t.item_tiles << " " << ms;
  write_cache_line(path, key, os.str());
}

// Batched plans: the whole-cube item size (bytes each workgroup moves) and
// one workgroup per item against persistent workgroups walking the list.
static spinsum_status autotune_batched(spinsum_plan_t P, const void* in, void* out,
                                       hipStream_t s, const char* cache_path,
                                       spinsum_tile_t* best, float* best_ms) {
  const void* const* ins = reinterpret_cast<const void* const*>(in);
  void* const* outs = reinterpret_cast<void* const*>(out);
  const int64_t keep_bytes = P->batch_item_bytes;
  const int keep_pers = P->batch_persistent;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
  bool have = false;
  int64_t win_bytes = 0;
  int win_pers = 0;
  float win_ms = 0;
  for (int pers = 0; pers <= 1; ++pers)
    for (int64_t kib : {8, 16, 24, 32, 40, 48, 64}) {
      P->batch_persistent = pers;
      if (build_batched(P, kib * 1024) != SPINSUM_OK || upload_tables(P) != SPINSUM_OK) continue;
      if (spinsum_exec_batched(P, ins, outs, s) != SPINSUM_OK) continue;  // warm-up
      float ms_min = 1e30f;
      bool ok = true;
      for (int r = 0; r < 3 && ok; ++r) {
        (void)hipEventRecord(e0, s);
        ok = spinsum_exec_batched(P, ins, outs, s) == SPINSUM_OK;
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms_min = std::min(ms_min, ms);
      }
      if (ok && (!have || ms_min < win_ms)) {
        have = true;
        win_bytes = kib * 1024;
        win_pers = pers;
        win_ms = ms_min;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->batch_persistent = have ? win_pers : keep_pers;
  spinsum_status st = build_batched(P, have ? win_bytes : keep_bytes);
  if (st == SPINSUM_OK) st = upload_tables(P);
  if (st != SPINSUM_OK) return st;
  if (best) {
    std::memset(best, 0, sizeof(*best));
    best->cubes_per_wg = (int)(P->batch_item_bytes / 1024);
    best->threads = 256;
    best->variant = P->batch_persistent;
  }
  if (best_ms) *best_ms = have ? win_ms : 0.0f;
  if (have && cache_path != nullptr && *cache_path) {
    std::ostringstream os;
    os << batched_key(*P) << " " << win_bytes / 1024 << " " << win_pers << " " << win_ms;
    write_cache_line(cache_path, batched_key(*P), os.str());
  }
  return have ? SPINSUM_OK : SPINSUM_ERR_UNSUPPORTED;
}

}  // namespace spinsum

using namespace spinsum;

extern "C" spinsum_status spinsum_autotune(spinsum_plan_t P, void* in, void* out, void* stream,
                                           const char* cache_path, spinsum_tile_t* best,
                                           float* best_ms) {
  if (P == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if (P->sub) return spinsum_autotune(P->sub, in, out, stream, cache_path, best, best_ms);
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  if (P->batched) {
    if (in == nullptr || out == nullptr) return SPINSUM_ERR_INVALID_ARG;
    return autotune_batched(P, in, out, (hipStream_t)stream, cache_path, best, best_ms);
  }
  if (P->pair) return SPINSUM_ERR_UNSUPPORTED;
  if (P->elems == 0) return SPINSUM_OK;
  hipStream_t s = (hipStream_t)stream;
  const int esz = elem_size(*P);
  const int n = P->n, d = P->d;
  int64_t cube_bytes = (int64_t)esz * P->inner;
  for (int m = 0; m < d; ++m) cube_bytes *= n;
  // candidates: kernel variant x tile edge (x cubes per workgroup)
  std::vector<spinsum_tile_t> shapes;
  for (int cpw = 1; cpw <= 64; cpw *= 2) {
    if (cpw * cube_bytes + 1024 > P->lds_limit || cpw > P->ncubes) break;
    if (cpw > 1 && cpw * cube_bytes > 96 * 1024) break;
    shapes.push_back({n, cpw, 256, 0, 0, 0});
  }
  for (int bl = n - 1; bl >= 2; --bl) {
    if (n % bl != 0) continue;
    if ((int64_t)bl * P->inner * esz < 32) continue;
    shapes.push_back({bl, 1, 256, 0, 0, 0});
    // work items packing several orbits: up to one and two largest orbits
    spinsum_tile_t probe{bl, 1, 256, 0, 0, 0};
    if (spinsum_plan_set_tile(P, &probe) != SPINSUM_OK) continue;
    const int mo = P->T.max_orbit_tiles;
    shapes.push_back({bl, 1, 256, 0, 0, mo});
    if (2 * mo <= kMaxGroupTiles) shapes.push_back({bl, 1, 256, 0, 0, 2 * mo});
  }
  std::vector<spinsum_tile_t> cands;
  for (const spinsum_tile_t& sh : shapes) {
    spinsum_tile_t t = sh;
    t.lds_pad = 0;
    t.variant = SPINSUM_VARIANT_DIRECT_LDS;
    for (int th : {256, 512, 1024}) {
      t.threads = th;
      cands.push_back(t);
    }
    t.threads = 256;
    t.variant = SPINSUM_VARIANT_LDS_PIPELINE;
    cands.push_back(t);
    for (int pad = 1; pad >= 0; --pad) {
      t.lds_pad = pad;
      t.variant = SPINSUM_VARIANT_REG_ONESHOT;
      cands.push_back(t);
      t.variant = SPINSUM_VARIANT_REG_PIPELINE;
      cands.push_back(t);
    }
  }
  spinsum_tile_t keep = P->tile;
  spinsum_tile_t win{};
  float win_ms = 0;
  bool have = false;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
  for (const spinsum_tile_t& t : cands) {
    if (spinsum_plan_set_tile(P, &t) != SPINSUM_OK) continue;
    if (spinsum_exec(P, in, out, stream) != SPINSUM_OK) continue;  // warm-up
    const int reps = 3;
    float ms_min = 1e30f;
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) {
      (void)hipEventRecord(e0, s);
      ok = spinsum_exec(P, in, out, stream) == SPINSUM_OK;
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    if (!ok) continue;
    if (!have || ms_min < win_ms) {
      have = true;
      win = P->tile;
      win_ms = ms_min;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  spinsum_status st = spinsum_plan_set_tile(P, have ? &win : &keep);
  if (st != SPINSUM_OK) return st;
  if (best) *best = P->tile;
  if (best_ms) *best_ms = have ? win_ms : 0.0f;
  if (have && cache_path != nullptr && *cache_path) cache_store(*P, cache_path, P->tile, win_ms);
  return have ? SPINSUM_OK : SPINSUM_ERR_UNSUPPORTED;
}
