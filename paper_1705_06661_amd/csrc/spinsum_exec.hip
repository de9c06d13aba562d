// spinsum_exec.hip -- exec / adjoint / batched / graph / copy entry points of
// the C-ABI of libspinsum (argument checks and dispatch to the per-dtype
// launchers).
#include <mutex>

#include "spinsum_device.h"

namespace spinsum {
namespace {

// Plain copy with the same 16-byte loads and non-temporal stores, one
// vector per thread: the achievable HBM ceiling for a read-once /
// write-once kernel.
__global__ void __launch_bounds__(kThreads) k_copy(const double* __restrict__ in,
                                                   double* __restrict__ out, int64_t nvec) {
  typedef double V __attribute__((ext_vector_type(2)));
  const V* src = reinterpret_cast<const V*>(in);
  V* dst = reinterpret_cast<V*>(out);
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < nvec) __builtin_nontemporal_store(src[i], dst + i);
}

template <typename T>
const void* pick_kernel(int d, int kind, int vw, bool chain, bool nts, int maxc) {
  if constexpr (sizeof(T) == 8) {
    if (d == 2) return pick_f64_d2(kind, vw, chain, nts, maxc);
    if (d == 3) return pick_f64_d3(kind, vw, chain, nts, maxc);
    return pick_f64_d4(kind, vw, chain, nts, maxc);
  } else {
    if (d == 2) return pick_f32_d2(kind, vw, chain, nts, maxc);
    if (d == 3) return pick_f32_d3(kind, vw, chain, nts, maxc);
    return pick_f32_d4(kind, vw, chain, nts, maxc);
  }
}

template <typename T>
const void* pick_batched(int d, int vw, bool persist) {
  if constexpr (sizeof(T) == 8) {
    if (d == 2) return pick_batched_f64_d2(vw, persist);
    if (d == 3) return pick_batched_f64_d3(vw, persist);
    return pick_batched_f64_d4(vw, persist);
  } else {
    if (d == 2) return pick_batched_f32_d2(vw, persist);
    if (d == 3) return pick_batched_f32_d3(vw, persist);
    return pick_batched_f32_d4(vw, persist);
  }
}

template <typename T>
const void* pick_pack(int d, bool pack, bool nts, bool persist) {
  if constexpr (sizeof(T) == 8) {
    if (d == 2) return pick_pack_f64_d2(pack, nts, persist);
    if (d == 3) return pick_pack_f64_d3(pack, nts, persist);
    return pick_pack_f64_d4(pack, nts, persist);
  } else {
    if (d == 2) return pick_pack_f32_d2(pack, nts, persist);
    if (d == 3) return pick_pack_f32_d3(pack, nts, persist);
    return pick_pack_f32_d4(pack, nts, persist);
  }
}

template <typename T>
const void* pick_cgrad(int d, bool split) {
  if constexpr (sizeof(T) == 8) {
    if (d == 2) return pick_cgrad_f64_d2(split);
    if (d == 3) return pick_cgrad_f64_d3(split);
    return pick_cgrad_f64_d4(split);
  } else {
    if (d == 2) return pick_cgrad_f32_d2(split);
    if (d == 3) return pick_cgrad_f32_d3(split);
    return pick_cgrad_f32_d4(split);
  }
}

spinsum_status hip_error(spinsum_plan_s* P, hipError_t e) {
  P->last_hip_error = (int)e;
  (void)hipGetLastError();
  return SPINSUM_ERR_HIP;
}

spinsum_status prepare_kernel(spinsum_plan_s* P, const void* k, size_t shmem) {
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return hip_error(P, e);
  }
  return SPINSUM_OK;
}

// Kernel, dynamic LDS and workgroup size of a plan's exec / adjoint launch
// (both launch the same kernel), and whether that kernel is persistent.
struct LaunchCfg {
  const void* k = nullptr;
  size_t shmem = 0;
  int threads = kThreads;
  int kind = 0;
  bool persistent = false;
};

template <typename T>
LaunchCfg exec_cfg(const spinsum_plan_s* P, bool chain) {
  const Tiling& Tl = P->T;
  const bool nts = Tl.nts != 0;
  LaunchCfg c;
  int kind = P->tile.variant;
  if (!nts && kind == SPINSUM_VARIANT_REG_PIPELINE) kind = SPINSUM_VARIANT_REG_ONESHOT;
  const int maxc = (kind == SPINSUM_VARIANT_REG_PIPELINE) ? (Tl.chunks_per_thread <= 8 ? 8 : 16) : 0;
  c.kind = kind;
  c.k = pick_kernel<T>(P->d, kind, Tl.vw, chain, nts, maxc);
  const size_t tile_bytes = ((size_t)Tl.lds_elems * sizeof(T) + 15) / 16 * 16;
  c.shmem = (size_t)Tl.lds_elems * sizeof(T);
  if (kind == SPINSUM_VARIANT_REG_PIPELINE || kind == SPINSUM_VARIANT_DIRECT_LDS)
    c.shmem = tile_bytes + (size_t)Tl.max_rep_cnt * 4;
  else if (kind == SPINSUM_VARIANT_LDS_PIPELINE)
    c.shmem = ((size_t)Tl.reps.size() * 4 + 15) / 16 * 16 + 2 * tile_bytes;
  c.threads = (kind == SPINSUM_VARIANT_DIRECT_LDS || kind == SPINSUM_VARIANT_LDS_PIPELINE)
                  ? P->tile.threads
                  : kThreads;
  c.persistent = (kind == SPINSUM_VARIANT_REG_PIPELINE || kind == SPINSUM_VARIANT_LDS_PIPELINE);
  return c;
}

template <typename T>
LaunchCfg batched_cfg(const spinsum_plan_s* P) {
  LaunchCfg c;
  c.persistent = P->batch_persistent != 0;
  c.k = pick_batched<T>(P->d, P->batch_vw, c.persistent);
  c.shmem = ((size_t)P->batch_lds_elems * sizeof(T) + 15) / 16 * 16 + (size_t)P->batch_rep_bytes;
  c.threads = kThreads;
  return c;
}

// Workgroups of a persistent launch: the occupancy of the kernel (taken
// when the plan's tables are made, see cache_occupancy) times the CUs,
// rounded down to a multiple of 8 (one share per XCD).
int64_t persistent_grid(const spinsum_plan_s* P, int64_t nitems) {
  int64_t g = (int64_t)std::max(1, P->occ_blocks) * P->num_cus;
  g = std::min<int64_t>(g, ((nitems + 7) / 8) * 8);
  return std::max<int64_t>(8, (g / 8) * 8);
}

// Which coefficients one launch applies: the pre-multiplied vector (forward
// or adjoint), every stage in registers (CHAIN), or one stage (the
// multi-pass form and the per-stage gradients).  offset: in elements of
// the plan's coefficient buffer (forward | adjoint | stages | adjoint
// stages, d! each).
struct CoefSel {
  size_t offset = 0;
  int nstages = 1;
  uint32_t sparse = 0;
  bool chain = false;
};

CoefSel coef_sel(const spinsum_plan_s* P, bool adjoint) {
  const int df = P->G.df;
  const int K = (int)P->stage_a.size();
  CoefSel c;
  if (P->flags & SPINSUM_FLAG_CHAIN_STAGES) {
    c.offset = 2 * (size_t)df + (adjoint ? (size_t)K * df : 0);
    c.nstages = K;
    c.sparse = adjoint ? P->sparse_adj : P->sparse_fwd;
    c.chain = true;
  } else {
    c.offset = adjoint ? (size_t)df : 0;
    c.sparse = P->sparse_expanded;
  }
  return c;
}

// Stage j in application order: of the forward chain (stage j) or of the
// adjoint chain (the inverse of stage K-1-j).
CoefSel stage_sel(const spinsum_plan_s* P, bool adjoint, int j) {
  const int df = P->G.df;
  const int K = (int)P->stage_a.size();
  CoefSel c;
  c.offset = 2 * (size_t)df + (adjoint ? (size_t)K * df : 0) + (size_t)j * df;
  const uint32_t m = adjoint ? P->sparse_adj : P->sparse_fwd;
  c.sparse = (j >= 32 || ((m >> j) & 1u) != 0u) ? 1u : 0u;
  return c;
}

template <typename T>
spinsum_status launch_exec(spinsum_plan_s* P, const void* in, void* out, hipStream_t stream,
                           const CoefSel& sel) {
  const Tiling& Tl = P->T;
  if (Tl.nitems <= 0) return SPINSUM_OK;
  const T* coef = reinterpret_cast<const T*>(P->d_mats);
  ExecArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.in = reinterpret_cast<const T*>(in);
  a.out = reinterpret_cast<T*>(out);
  a.orbits = reinterpret_cast<const GroupDev*>(P->d_orbits);
  a.reps = reinterpret_cast<const uint32_t*>(P->d_reps);
  a.coef = coef + sel.offset;
  a.nstages = sel.nstages;
  a.sparse = sel.sparse;
  a.g = Tl.g;
  a.nitems = Tl.nitems;
  a.reverse = (P->flags & SPINSUM_FLAG_REVERSE_ORDER) ? 1 : 0;
  a.nt_loads = Tl.ntl;
  // kernel variant chosen by the planner (see spinsum_tile_t.variant)
  const LaunchCfg c = exec_cfg<T>(P, sel.chain);
  a.lds_tile_bytes = (int32_t)(((size_t)Tl.lds_elems * sizeof(T) + 15) / 16 * 16);
  a.nreps = (int32_t)Tl.reps.size();
  spinsum_status st = prepare_kernel(P, c.k, c.shmem);
  if (st != SPINSUM_OK) return st;
  int64_t grid;
  if (c.persistent) {
    grid = persistent_grid(P, Tl.nitems);
    a.xcd_per = (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) ? 0 : (Tl.nitems + 7) / 8;
  } else if (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) {
    a.xcd_per = 0;
    grid = Tl.nitems;
  } else {
    a.xcd_per = (Tl.nitems + 7) / 8;
    grid = a.xcd_per * 8;
  }
  void* kargs[] = {&a};
  hipError_t e = hipLaunchKernel(c.k, dim3((unsigned)grid), dim3(c.threads), kargs, c.shmem, stream);
  if (e != hipSuccess) return hip_error(P, e);
  return SPINSUM_OK;
}

// Index-pair form: one tile orbit of one pair block per workgroup.
template <typename T>
spinsum_status launch_pair(spinsum_plan_s* P, const void* in, void* out, hipStream_t stream,
                           const CoefSel& sel) {
  const Tiling& Tl = P->T;
  if (Tl.nitems <= 0) return SPINSUM_OK;
  const bool chain = sel.chain;
  const bool nts = Tl.nts != 0;
  const T* coef = reinterpret_cast<const T*>(P->d_mats);
  PairArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.in = reinterpret_cast<const T*>(in);
  a.out = reinterpret_cast<T*>(out);
  a.orbits = reinterpret_cast<const uint64_t*>(P->d_orbits);
  a.reps = reinterpret_cast<const uint32_t*>(P->d_reps);
  a.coef = coef + sel.offset;
  a.nstages = sel.nstages;
  a.sparse = sel.sparse;
  a.g = Tl.g;
  a.pg = P->pg;
  a.nitems = Tl.nitems;
  a.reverse = (P->flags & SPINSUM_FLAG_REVERSE_ORDER) ? 1 : 0;
  a.lds_tile_bytes = (int32_t)(((size_t)Tl.lds_elems * sizeof(T) + 15) / 16 * 16);
  const void* k = pick_kernel<T>(P->d, 5, Tl.vw, chain, nts, 0);
  const size_t shmem = (size_t)a.lds_tile_bytes + (size_t)Tl.max_rep_cnt * 4;
  spinsum_status st = prepare_kernel(P, k, shmem);
  if (st != SPINSUM_OK) return st;
  int64_t grid;
  if (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) {
    a.xcd_per = 0;
    grid = Tl.nitems;
  } else {
    a.xcd_per = (Tl.nitems + 7) / 8;
    grid = a.xcd_per * 8;
  }
  void* kargs[] = {&a};
  hipError_t e =
      hipLaunchKernel(k, dim3((unsigned)grid), dim3(P->tile.threads), kargs, shmem, stream);
  if (e != hipSuccess) return hip_error(P, e);
  return SPINSUM_OK;
}

template <typename T>
spinsum_status launch_batched(spinsum_plan_s* P, const void* const* in, void* const* out,
                              hipStream_t stream) {
  if (P->items.empty()) return SPINSUM_OK;
  BatchArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.in = reinterpret_cast<const T* const*>(in);
  a.out = reinterpret_cast<T* const*>(out);
  a.orbits = reinterpret_cast<const GroupDev*>(P->d_orbits);
  a.reps = reinterpret_cast<const uint32_t*>(P->d_reps);
  a.coef = reinterpret_cast<const T*>(P->d_mats);
  a.blocks = reinterpret_cast<const BatchBlock*>(P->d_blocks);
  a.items = reinterpret_cast<const BatchItem*>(P->d_items);
  a.nitems = (int64_t)P->items.size();
  a.lds_tile_bytes = (int32_t)(((size_t)P->batch_lds_elems * sizeof(T) + 15) / 16 * 16);
  a.sparse = P->sparse_expanded;
  const LaunchCfg c = batched_cfg<T>(P);
  const void* k = c.k;
  const size_t shmem = c.shmem;
  spinsum_status st = prepare_kernel(P, k, shmem);
  if (st != SPINSUM_OK) return st;
  int64_t grid;
  if (c.persistent) {
    grid = persistent_grid(P, a.nitems);
    a.xcd_per = (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) ? 0 : (a.nitems + 7) / 8;
  } else if (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) {
    a.xcd_per = 0;
    grid = a.nitems;
  } else {
    a.xcd_per = (a.nitems + 7) / 8;
    grid = a.xcd_per * 8;
  }
  void* kargs[] = {&a};
  hipError_t e = hipLaunchKernel(k, dim3((unsigned)grid), dim3(kThreads), kargs, shmem, stream);
  if (e != hipSuccess) return hip_error(P, e);
  return SPINSUM_OK;
}

template <typename T>
spinsum_status occupancy_of(spinsum_plan_s* P) {
  P->occ_blocks = 1;
  if (P->pair) return SPINSUM_OK;
  const LaunchCfg c =
      P->batched ? batched_cfg<T>(P) : exec_cfg<T>(P, (P->flags & SPINSUM_FLAG_CHAIN_STAGES) != 0);
  if (!c.persistent || c.k == nullptr) return SPINSUM_OK;
  spinsum_status st = prepare_kernel(P, c.k, c.shmem);
  if (st != SPINSUM_OK) return st;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c.k, c.threads, c.shmem);
  if (e != hipSuccess) return hip_error(P, e);
  P->occ_blocks = std::max(1, per_cu);
  return SPINSUM_OK;
}

// Workgroups per CU of the persistent unpacking kernel.
template <typename T>
spinsum_status unpack_occupancy_of(spinsum_plan_s* P) {
  P->pk_persist_blocks = 1;
  if (!P->pk_persist) return SPINSUM_OK;
  const void* k = pick_pack<T>(P->d, false, P->Tu.nts != 0, true);
  if (k == nullptr) return SPINSUM_ERR_UNSUPPORTED;
  const size_t shmem = ((size_t)P->Tu.lds_elems * sizeof(T) + 15) / 16 * 16;
  spinsum_status st = prepare_kernel(P, k, shmem);
  if (st != SPINSUM_OK) return st;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, P->pk_threads, shmem);
  if (e != hipSuccess) return hip_error(P, e);
  P->pk_persist_blocks = std::max(1, per_cu);
  return SPINSUM_OK;
}

spinsum_status check_device(spinsum_plan_s* P) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(P, e);
  if (dev != P->device) return SPINSUM_ERR_INVALID_ARG;
  return SPINSUM_OK;
}

spinsum_status check_tensor_args(spinsum_plan_s* P, const void* in, const void* out) {
  if (P == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if (P->batched) return SPINSUM_ERR_INVALID_ARG;
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  if (P->elems == 0) return SPINSUM_OK;
  if (in == nullptr || out == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if ((((uintptr_t)in) | ((uintptr_t)out)) & 15u) return SPINSUM_ERR_MISALIGNED;
  if (P->inplace) {
    if (in != out) return SPINSUM_ERR_INVALID_ARG;
  } else {
    const uintptr_t bytes = (uintptr_t)P->elems * (uintptr_t)elem_size(*P);
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a < b + bytes && b < a + bytes) return SPINSUM_ERR_ALIASING;
  }
  return check_device(P);
}

}  // namespace

// Occupancy of a persistent exec kernel, taken whenever a plan's tables are
// made (plan creation, spinsum_plan_set_tile, the autotuner), so that exec
// only reads the plan.
spinsum_status cache_occupancy(spinsum_plan_s* P) {
  if (!P->has_dev) return SPINSUM_OK;
  spinsum_status st = P->dtype == SPINSUM_F32 ? occupancy_of<float>(P) : occupancy_of<double>(P);
  if (st != SPINSUM_OK) return st;
  return P->dtype == SPINSUM_F32 ? unpack_occupancy_of<float>(P) : unpack_occupancy_of<double>(P);
}

}  // namespace spinsum

using namespace spinsum;

namespace spinsum {
namespace {

// One launch of the plan's kernel with the coefficients `sel`.
spinsum_status launch_any(spinsum_plan_s* P, const void* in, void* out, hipStream_t stream,
                          const CoefSel& sel) {
  if (P->pair) {
    if (P->dtype == SPINSUM_F32) return launch_pair<float>(P, in, out, stream, sel);
    return launch_pair<double>(P, in, out, stream, sel);
  }
  if (P->dtype == SPINSUM_F32) return launch_exec<float>(P, in, out, stream, sel);
  return launch_exec<double>(P, in, out, stream, sel);
}

// Stages j0 .. j1-1 of the forward or adjoint chain, one launch each: the
// first from `in` to `out`, the others in place on `out` (every launch
// reads a whole tile orbit before writing it, so a stage can run in place
// on any buffer).
spinsum_status launch_stages(spinsum_plan_s* P, const void* in, void* out, hipStream_t stream,
                             bool adjoint, int j0, int j1) {
  for (int j = j0; j < j1; ++j) {
    spinsum_status st = launch_any(P, j == j0 ? in : out, out, stream, stage_sel(P, adjoint, j));
    if (st != SPINSUM_OK) return st;
  }
  return SPINSUM_OK;
}

// exec / adjoint: one launch (the pre-multiplied operator, or every stage
// in registers), or with SPINSUM_FLAG_MULTI_PASS one launch per stage
// through the output buffer (Alg. 3).
spinsum_status run(spinsum_plan_s* P, const void* in, void* out, hipStream_t stream,
                   bool adjoint) {
  if (P->sub) return run(P->sub, in, out, stream, adjoint);  // the moved axes alone
  if (P->flags & SPINSUM_FLAG_MULTI_PASS)
    return launch_stages(P, in, out, stream, adjoint, 0, (int)P->stage_a.size());
  return launch_any(P, in, out, stream, coef_sel(P, adjoint));
}

}  // namespace
}  // namespace spinsum

extern "C" spinsum_status spinsum_exec(spinsum_plan_t P, const void* in, void* out, void* stream) {
  spinsum_status st = check_tensor_args(P, in, out);
  if (st != SPINSUM_OK || P->elems == 0) return st;
  return run(P, in, out, (hipStream_t)stream, false);
}

extern "C" spinsum_status spinsum_adjoint(spinsum_plan_t P, const void* grad_out, void* grad_in,
                                          void* stream) {
  spinsum_status st = check_tensor_args(P, grad_out, grad_in);
  if (st != SPINSUM_OK || P->elems == 0) return st;
  return run(P, grad_out, grad_in, (hipStream_t)stream, true);
}

namespace spinsum {
namespace {

template <typename T>
spinsum_status launch_cgrad(spinsum_plan_s* P, const void* x, const void* g, double* grad,
                            double* part, hipStream_t stream) {
  // one tile buffer on the plan's tiling where it allows (k_cgrad_split),
  // else both tensors in LDS on the packed tiling where the plan has one
  // (see build_cgrad_tiling)
  const bool split = P->cg_split;
  const bool packed = P->cg_pack && !split;
  const Tiling& Tl = packed ? P->Tc : P->T;
  CGradArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.x = reinterpret_cast<const T*>(x);
  a.gr = reinterpret_cast<const T*>(g);
  a.grad = part;
  a.orbits = reinterpret_cast<const GroupDev*>(packed ? P->d_cg_orbits : P->d_orbits);
  a.reps = reinterpret_cast<const uint32_t*>(packed ? P->d_cg_reps : P->d_reps);
  a.g = Tl.g;
  a.nitems = Tl.nitems;
  a.lds_tile_bytes = (int32_t)(((size_t)Tl.lds_elems * sizeof(T) + 15) / 16 * 16);
  const int df = P->G.df;
  // LDS: x tiles | gradient tiles (k_cgrad only) | representative lists;
  // the partial sums of the waves reuse it at the end
  const size_t shmem = std::max<size_t>((split ? 1 : 2) * (size_t)a.lds_tile_bytes +
                                            (size_t)Tl.max_rep_cnt * 4,
                                        (size_t)(kThreads / 64) * df * sizeof(double));
  if ((int64_t)shmem > P->lds_limit) return SPINSUM_ERR_UNSUPPORTED;
  const void* k = pick_cgrad<T>(P->d, split);
  spinsum_status st = prepare_kernel(P, k, shmem);
  if (st != SPINSUM_OK) return st;
  hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(kThreads), 0, stream, a.grad, kGradSlots * df);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(P, e);
  int64_t grid;
  if (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) {
    a.xcd_per = 0;
    grid = Tl.nitems;
  } else {
    a.xcd_per = (Tl.nitems + 7) / 8;
    grid = a.xcd_per * 8;
  }
  void* kargs[] = {&a};
  e = hipLaunchKernel(k, dim3((unsigned)grid), dim3(kThreads), kargs, shmem, stream);
  if (e != hipSuccess) return hip_error(P, e);
  hipLaunchKernelGGL(k_grad_reduce, dim3(df), dim3(kThreads), 0, stream,
                     (const double*)a.grad, grad, df);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(P, e);
  return SPINSUM_OK;
}

}  // namespace
}  // namespace spinsum

namespace spinsum {
namespace {

// The coefficient gradient's partial sums for callers that cannot allocate
// (spinsum_coef_grad_noalloc): one array per GPU for the life of the
// process, shared by every call on that GPU.  In host code `scratch` only
// names the symbol; its device address is taken once per device
// (scratch_on_device) and that address is what the kernels receive.
constexpr int kScratchDoubles = kGradSlots * kMaxDF;  // 384 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (the current device, which
// check_device has matched to the plan's).
spinsum_status scratch_on_device(spinsum_plan_s* P, double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(P, e);
  if (dev < 0 || dev >= kMaxDevices) return SPINSUM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return hip_error(P, e != hipSuccess ? e : hipErrorInvalidSymbol);
    scratch_ptr[dev] = reinterpret_cast<double*>(ptr);
  }
  *out = scratch_ptr[dev];
  return SPINSUM_OK;
}

// spinsum_coef_grad with the partial sums in `part` (kGradSlots x d!
// doubles) or, for part == nullptr, in this device's `scratch`.
spinsum_status coef_grad_impl(spinsum_plan_s* P, const void* x, const void* g, double* grad,
                              bool use_scratch, void* stream) {
  if (P == nullptr || P->batched || grad == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  if (((uintptr_t)grad) & 7u) return SPINSUM_ERR_MISALIGNED;
  if (P->pair) return SPINSUM_ERR_UNSUPPORTED;
  if (P->elems == 0) {
    spinsum_status st = check_device(P);
    if (st != SPINSUM_OK) return st;
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(kThreads), 0, (hipStream_t)stream, grad, P->G.df);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPINSUM_OK : hip_error(P, e);
  }
  if (x == nullptr || g == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if ((((uintptr_t)x) | ((uintptr_t)g)) & 15u) return SPINSUM_ERR_MISALIGNED;
  spinsum_status st = check_device(P);
  if (st != SPINSUM_OK) return st;
  // the direct-LDS layout: whole cubes, or tiles whose rows are whole
  // 16-byte chunks, unpadded
  const Tiling& Tl = P->T;
  const bool whole = Tl.g.bl == Tl.g.n;
  const bool rows = Tl.vw * elem_size(*P) == 16;
  if (P->tile.lds_pad != 0 || !(whole || rows)) return SPINSUM_ERR_UNSUPPORTED;
  double* part = reinterpret_cast<double*>(P->d_grad_part);
  if (use_scratch) {
    if ((int64_t)kGradSlots * P->G.df > kScratchDoubles) return SPINSUM_ERR_UNSUPPORTED;
    st = scratch_on_device(P, &part);
    if (st != SPINSUM_OK) return st;
  }
  if (P->dtype == SPINSUM_F32) return launch_cgrad<float>(P, x, g, grad, part, (hipStream_t)stream);
  return launch_cgrad<double>(P, x, g, grad, part, (hipStream_t)stream);
}

}  // namespace
}  // namespace spinsum

extern "C" spinsum_status spinsum_coef_grad(spinsum_plan_t P, const void* x, const void* g,
                                            double* grad, void* stream) {
  return coef_grad_impl(P, x, g, grad, false, stream);
}

extern "C" spinsum_status spinsum_coef_grad_stages(spinsum_plan_t P, const void* x, const void* g,
                                                   double* grad, void* work_u, void* work_h,
                                                   void* stream) {
  if (P == nullptr || P->batched || grad == nullptr) return SPINSUM_ERR_INVALID_ARG;
  const int K = (int)P->stage_a.size();
  const int df = P->G.df;
  hipStream_t s = (hipStream_t)stream;
  if (K == 1 || P->elems == 0) return coef_grad_impl(P, x, g, grad, false, stream);
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  if (P->pair) return SPINSUM_ERR_UNSUPPORTED;
  if (x == nullptr || g == nullptr || work_u == nullptr || work_h == nullptr)
    return SPINSUM_ERR_INVALID_ARG;
  if ((((uintptr_t)x) | ((uintptr_t)g) | ((uintptr_t)work_u) | ((uintptr_t)work_h)) & 15u)
    return SPINSUM_ERR_MISALIGNED;
  const uintptr_t bytes = (uintptr_t)P->elems * (uintptr_t)elem_size(*P);
  auto overlap = [&](const void* p, const void* q) {
    const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + bytes && b < a + bytes;
  };
  if (overlap(work_u, work_h) || overlap(work_u, x) || overlap(work_u, g) || overlap(work_h, x) ||
      overlap(work_h, g))
    return SPINSUM_ERR_ALIASING;
  for (int k = 0; k < K; ++k) {
    // u = S_{k-1} ... S_1 x (stages 0 .. k-1), h = S_{k+1}^T ... S_K^T g
    // (adjoint chain positions 0 .. K-2-k)
    const void* u = x;
    const void* h = g;
    spinsum_status st;
    if (k > 0) {
      st = launch_stages(P, x, work_u, s, false, 0, k);
      if (st != SPINSUM_OK) return st;
      u = work_u;
    }
    if (k < K - 1) {
      st = launch_stages(P, g, work_h, s, true, 0, K - 1 - k);
      if (st != SPINSUM_OK) return st;
      h = work_h;
    }
    st = coef_grad_impl(P, u, h, grad + (size_t)k * df, false, stream);
    if (st != SPINSUM_OK) return st;
  }
  return SPINSUM_OK;
}

extern "C" spinsum_status spinsum_coef_grad_noalloc(spinsum_plan_t P, const void* x,
                                                    const void* g, double* grad, void* stream) {
  return coef_grad_impl(P, x, g, grad, true, stream);
}

namespace spinsum {
namespace {

// C(n, d), or -1 beyond 2^62.
int64_t ncomb_of(int n, int d) {
  int64_t r = 1;
  for (int k = 0; k < d; ++k) {
    if (r > ((int64_t)1 << 62) / std::max(1, n - k)) return -1;
    r = r * (n - k) / (k + 1);
  }
  return r;
}

template <typename T>
spinsum_status launch_pack(spinsum_plan_s* P, const void* full, void* packed, bool pack,
                           hipStream_t stream) {
  // unpacking on its own tiling where the plan has one (the largest items
  // that fit a CU, see build_unpack_tiling); packing on the plan's
  const bool own = !pack && P->pk_own;
  const Tiling& Tl = own ? P->Tu : P->T;
  if (Tl.nitems <= 0) return SPINSUM_OK;
  PackArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  if (pack) {
    a.full_in = reinterpret_cast<const T*>(full);
    a.packed_out = reinterpret_cast<T*>(packed);
  } else {
    a.full_out = reinterpret_cast<T*>(const_cast<void*>(full));
    a.packed_in = reinterpret_cast<const T*>(packed);
  }
  a.orbits = reinterpret_cast<const GroupDev*>(own ? P->d_pk_orbits : P->d_orbits);
  // packing writes one packed value per representative: in lexicographic
  // order the lanes of a wave write neighbouring entries (unpacking reads
  // them, and gains more from the bank-spreading order of its LDS scatter)
  a.reps = reinterpret_cast<const uint32_t*>(
      own ? P->d_pk_reps : (pack && P->d_reps_lex ? P->d_reps_lex : P->d_reps));
  a.coef = reinterpret_cast<const T*>(P->d_mats);  // the pre-multiplied forward vector
  a.g = Tl.g;
  a.nitems = Tl.nitems;
  a.ncomb = ncomb_of(P->n, P->d);
  a.lds_tile_bytes = (int32_t)(((size_t)Tl.lds_elems * sizeof(T) + 15) / 16 * 16);
  // persistently where the plan allows it: an occupancy-sized grid shared
  // among the item templates in proportion to their tiles, each workgroup
  // walking its XCD's range of cubes (no representative lists in LDS: every
  // thread keeps its own units)
  const bool persist = own && P->pk_persist && !(P->flags & SPINSUM_FLAG_NO_XCD_REMAP);
  const void* k = pick_pack<T>(P->d, pack, Tl.nts != 0, persist);
  const size_t shmem =
      (size_t)a.lds_tile_bytes + (persist ? (size_t)0 : (size_t)Tl.max_rep_cnt * 4);
  spinsum_status st = prepare_kernel(P, k, shmem);
  if (st != SPINSUM_OK) return st;
  int64_t grid;
  if (persist) {
    a.xcd_per = (P->ncubes + 7) / 8;
    const int nt = (int)Tl.groups.size();
    const bool whole = Tl.g.bl == Tl.g.n;
    int64_t tiles = 0;
    for (const GroupDev& gd : Tl.groups) tiles += whole ? 1 : gd.ntiles;
    const int64_t g8 = (int64_t)std::max(1, P->pk_persist_blocks) * P->num_cus / 8;
    a.ntmpl = nt;
    a.tmpl_wg[0] = 0;
    for (int t = 0; t < nt; ++t) {
      const int64_t share = (g8 * (whole ? 1 : Tl.groups[t].ntiles) + tiles / 2) / std::max<int64_t>(1, tiles);
      const int64_t w8 = std::min<int64_t>(std::max<int64_t>(1, share), a.xcd_per);
      a.tmpl_wg[t + 1] = a.tmpl_wg[t] + (int32_t)(8 * w8);
    }
    grid = a.tmpl_wg[nt];
  } else if (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) {
    a.xcd_per = 0;
    grid = Tl.nitems;
  } else {
    a.xcd_per = (Tl.nitems + 7) / 8;
    grid = a.xcd_per * 8;
  }
  void* kargs[] = {&a};
  hipError_t e = hipLaunchKernel(k, dim3((unsigned)grid), dim3(own ? P->pk_threads : P->tile.threads),
                                 kargs, shmem, stream);
  if (e != hipSuccess) return hip_error(P, e);
  return SPINSUM_OK;
}

spinsum_status pack_impl(spinsum_plan_s* P, const void* full, void* packed, bool pack,
                         void* stream) {
  if (P == nullptr || P->batched) return SPINSUM_ERR_INVALID_ARG;
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  if (P->pair) return SPINSUM_ERR_UNSUPPORTED;
  if (P->elems == 0) return check_device(P);
  if (full == nullptr || packed == nullptr) return SPINSUM_ERR_INVALID_ARG;
  const int esz = elem_size(*P);
  if ((((uintptr_t)full) & 15u) || (((uintptr_t)packed) & (uintptr_t)(esz - 1)))
    return SPINSUM_ERR_MISALIGNED;
  const int64_t ncomb = ncomb_of(P->n, P->d);
  if (ncomb < 0 || P->n >= (1 << 16)) return SPINSUM_ERR_UNSUPPORTED;
  const uintptr_t fbytes = (uintptr_t)P->elems * (uintptr_t)esz;
  const uintptr_t pbytes = (uintptr_t)(P->ncubes * ncomb * P->inner) * (uintptr_t)esz;
  const uintptr_t f = (uintptr_t)full, q = (uintptr_t)packed;
  if (pbytes > 0 && f < q + pbytes && q < f + fbytes) return SPINSUM_ERR_ALIASING;
  spinsum_status st = check_device(P);
  if (st != SPINSUM_OK) return st;
  // the tiles of the whole group, in the direct-LDS layout
  const Tiling& Tl = P->T;
  const bool whole = Tl.g.bl == Tl.g.n;
  const bool rows = Tl.vw * esz == 16;
  if (P->tile.lds_pad != 0 || !(whole || rows)) return SPINSUM_ERR_UNSUPPORTED;
  if (P->dtype == SPINSUM_F32) return launch_pack<float>(P, full, packed, pack, (hipStream_t)stream);
  return launch_pack<double>(P, full, packed, pack, (hipStream_t)stream);
}

}  // namespace
}  // namespace spinsum

extern "C" spinsum_status spinsum_unpack(spinsum_plan_t P, const void* packed, void* full,
                                         void* stream) {
  return pack_impl(P, full, const_cast<void*>(packed), false, stream);
}

extern "C" spinsum_status spinsum_pack(spinsum_plan_t P, const void* full, void* packed,
                                       void* stream) {
  return pack_impl(P, full, packed, true, stream);
}

extern "C" spinsum_status spinsum_exec_batched(spinsum_plan_t P, const void* const* in,
                                               void* const* out, void* stream) {
  if (P == nullptr || !P->batched) return SPINSUM_ERR_INVALID_ARG;
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  if (P->items.empty()) return SPINSUM_OK;
  if (in == nullptr || out == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if ((((uintptr_t)in) | ((uintptr_t)out)) & 7u) return SPINSUM_ERR_MISALIGNED;
  spinsum_status st = check_device(P);
  if (st != SPINSUM_OK) return st;
  if (P->dtype == SPINSUM_F32) return launch_batched<float>(P, in, out, (hipStream_t)stream);
  return launch_batched<double>(P, in, out, (hipStream_t)stream);
}

struct spinsum_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" spinsum_status spinsum_graph_create(spinsum_plan_t P, const void* const* in,
                                               void* const* out, spinsum_graph_t* graph) {
  if (P == nullptr || graph == nullptr) return SPINSUM_ERR_INVALID_ARG;
  *graph = nullptr;
  if (!P->has_dev) return SPINSUM_ERR_NO_DEVICE;
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_error(P, e);
  spinsum_graph_s* G = new (std::nothrow) spinsum_graph_s();
  if (!G) {
    (void)hipStreamDestroy(s);
    return SPINSUM_ERR_OUT_OF_MEMORY;
  }
  spinsum_status st = SPINSUM_OK;
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    if (P->batched)
      st = spinsum_exec_batched(P, in, out, s);
    else
      st = spinsum_exec(P, (const void*)in, (void*)out, s);
    hipError_t e2 = hipStreamEndCapture(s, &G->graph);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess && st == SPINSUM_OK) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(s);
  if (e != hipSuccess || st != SPINSUM_OK) {
    if (e != hipSuccess) {
      P->last_hip_error = (int)e;
      (void)hipGetLastError();
    }
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return st != SPINSUM_OK ? st : SPINSUM_ERR_HIP;
  }
  *graph = G;
  return SPINSUM_OK;
}

extern "C" spinsum_status spinsum_graph_launch(spinsum_graph_t G, void* stream) {
  if (G == nullptr || G->exec == nullptr) return SPINSUM_ERR_INVALID_ARG;
  hipError_t e = hipGraphLaunch(G->exec, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
  return SPINSUM_OK;
}

extern "C" void spinsum_graph_destroy(spinsum_graph_t G) {
  if (!G) return;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  delete G;
}

extern "C" spinsum_status spinsum_stream_copy(const void* in, void* out, int64_t nbytes,
                                              void* stream) {
  if (nbytes < 0 || (nbytes % 16) != 0) return SPINSUM_ERR_INVALID_ARG;
  if (nbytes == 0) return SPINSUM_OK;
  if (in == nullptr || out == nullptr) return SPINSUM_ERR_INVALID_ARG;
  if ((((uintptr_t)in) | ((uintptr_t)out)) & 15u) return SPINSUM_ERR_MISALIGNED;
  const int64_t nvec = nbytes / 16;
  const int64_t grid = (nvec + kThreads - 1) / kThreads;
  if (grid >= (1ll << 31)) return SPINSUM_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(kThreads), 0, (hipStream_t)stream,
                     (const double*)in, (double*)out, nvec);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPINSUM_OK : SPINSUM_ERR_HIP;
}
