// spinsum_kernels.hip -- gfx950 kernels of libspinsum and the exec entry
// points of the C-ABI.
//
// One workgroup processes one work item: a run of whole spectator cubes, or
// one tile orbit {sigma . B} of one cube (the macro-kernel of Alg. 5b/6).
//   1. load : every tile of the item is read from HBM once, with 16-byte
//             vector loads along the fastest (stride-one) axis, into LDS
//             (padded strides against bank conflicts);
//   2. combine: each thread takes element-orbit representatives x and reads
//             v_sigma = tile[sigma . x] for all sigma in S_d from LDS, forms
//             w = M v in registers (M the d! x d! orbit matrix of the
//             operator, or the product of the per-stage matrices applied one
//             after the other) and writes w_tau to tile[tau . x];
//   3. store: the tiles are written back once, 16-byte vector stores,
//             non-temporal by default (Sec. 4.6.3), to the same places
//             (in place, Sec. 4.6.5) or to the output tensor.
// Every element belongs to exactly one item, and inside an item to the
// element orbit of exactly one representative, so the in-place form needs
// only the two workgroup barriers.  The work is HBM-bound (0.75 flop/byte
// in 3D, 3 flop/byte in 4D): no matrix cores are used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "spinsum_plan_host.h"

namespace spinsum {
namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

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

template <typename T>
struct ExecArgs {
  const T* in;
  T* out;
  const OrbitDev* orbits;
  const uint32_t* reps;
  const T* mats;
  Geom g;
  int64_t nitems;
  int64_t xcd_per;  // > 0: items grouped per XCD
  int32_t nmats;
  int32_t reverse;
  int32_t nt;
  int32_t pad;
};

template <typename T>
struct BatchArgs {
  const T* const* in;
  T* const* out;
  const OrbitDev* orbits;
  const uint32_t* reps;
  const T* mats;
  const BatchBlock* blocks;
  const BatchItem* items;
  int64_t nitems;
  int32_t nt;
  int32_t pad;
};

template <typename T, int D, bool CHAIN>
__device__ __forceinline__ void combine(const T* __restrict__ mats, int nmats, T (&v)[Fact<D>::v],
                                        T (&w)[Fact<D>::v]) {
  constexpr int DF = Fact<D>::v;
  if constexpr (!CHAIN) {
#pragma unroll
    for (int t = 0; t < DF; ++t) {
      T acc = T(0);
#pragma unroll
      for (int s = 0; s < DF; ++s) acc = __builtin_fma(mats[t * DF + s], v[s], acc);
      w[t] = acc;
    }
  } else {
    for (int k = 0; k < nmats; ++k) {
      const T* Mk = mats + k * DF * DF;
#pragma unroll
      for (int t = 0; t < DF; ++t) {
        T acc = T(0);
#pragma unroll
        for (int s = 0; s < DF; ++s) acc = __builtin_fma(Mk[t * DF + s], v[s], acc);
        w[t] = acc;
      }
#pragma unroll
      for (int t = 0; t < DF; ++t) v[t] = w[t];
    }
    if (nmats == 0) {
#pragma unroll
      for (int t = 0; t < DF; ++t) w[t] = v[t];
    }
  }
}

template <typename T, int D, int VW, bool CHAIN, bool NTS>
__device__ __forceinline__ void run_item(const Geom& g, const OrbitDev* __restrict__ od,
                                         const uint32_t* __restrict__ reps,
                                         const T* __restrict__ mats, int nmats, const T* src,
                                         T* dst, int64_t cube0, int ncub, T* lds, int32_t* tinfo) {
  constexpr int DF = Fact<D>::v;
  typedef typename VecT<T, VW>::type V;
  const int tid = threadIdx.x;
  const int ntiles = od->ntiles;
  const bool ragged = od->ragged != 0;
  if (tid < ntiles) {
    tinfo[tid] = od->tile_off[tid];
    tinfo[kMaxDF + tid] = od->tile_ext[tid];
  }
  __syncthreads();

  const uint32_t nchunks = (uint32_t)ncub * (uint32_t)ntiles * (uint32_t)g.rows * (uint32_t)g.vpr;
  const T* sbase = src + cube0 * g.cube_elems;
  T* dbase = dst + cube0 * g.cube_elems;

  // 1. load every tile of the item into LDS
  for (uint32_t c0 = tid; c0 < nchunks; c0 += kUnroll * kThreads) {
    V buf[kUnroll];
    int lo[kUnroll];
    bool ok[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint32_t c = c0 + u * kThreads;
      int64_t go = 0;
      lo[u] = 0;
      ok[u] = (c < nchunks) && chunk_addr<D, VW>(g, c, ntiles, tinfo, tinfo + kMaxDF, ragged, &go, &lo[u]);
      if (ok[u]) buf[u] = *reinterpret_cast<const V*>(sbase + go);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ok[u]) {
#pragma unroll
        for (int k = 0; k < VW; ++k) lds[lo[u] + k] = vget<V, T, VW>(buf[u], k);
      }
  }
  __syncthreads();

  // 2. combine every element orbit in registers
  {
    int32_t sb[DF];
#pragma unroll
    for (int r = 0; r < DF; ++r) sb[r] = od->slot_base[r];
    const uint32_t rep_cnt = (uint32_t)od->rep_cnt;
    const uint32_t nrep = (uint32_t)ncub * rep_cnt;
    const uint32_t* rp = reps + od->rep_off;
    const FastDiv fdr = od->fd_rep;
    for (uint32_t i = tid; i < nrep; i += kThreads) {
      uint32_t ci = (ncub == 1) ? 0u : fdiv(i, fdr);
      uint32_t ri = i - ci * rep_cnt;
      uint32_t pk = rp[ri];
      int l[D];
#pragma unroll
      for (int m = 0; m < D; ++m) l[m] = (int)((pk >> (8 * m)) & 255u);
      const int base = (int)ci * g.cube_lds;
      int addr[DF];
      T v[DF];
      T w[DF];
#pragma unroll
      for (int r = 0; r < DF; ++r) {
        addr[r] = orbit_lds_addr<D>(g, base, sb, r, l);
        v[r] = lds[addr[r]];
      }
      // keep the orbit matrix in the scalar cache: without this barrier the
      // compiler hoists all d!^2 coefficients out of the loop into VGPRs
      asm volatile("" ::: "memory");
      combine<T, D, CHAIN>(mats, nmats, v, w);
#pragma unroll
      for (int r = 0; r < DF; ++r) lds[addr[r]] = w[r];
    }
  }
  __syncthreads();

  // 3. store every tile of the item
  for (uint32_t c0 = tid; c0 < nchunks; c0 += kUnroll * kThreads) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      uint32_t c = c0 + u * kThreads;
      int64_t go = 0;
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

template <typename T, int D, int VW, bool CHAIN, bool NTS>
__global__ void __launch_bounds__(kThreads) k_exec(const ExecArgs<T> a) {
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
  if (g.bl == g.n) {
    cube0 = item * g.cpw;
    orbit = 0;
    int64_t left = g.ncubes - cube0;
    ncub = (int)(left < g.cpw ? left : g.cpw);
  } else {
    uint32_t q = fdiv((uint32_t)item, g.fd_norbits);
    cube0 = q;
    orbit = (int)((uint32_t)item - q * (uint32_t)g.norbits);
    ncub = 1;
  }
  run_item<T, D, VW, CHAIN, NTS>(g, a.orbits + orbit, a.reps, a.mats, a.nmats, a.in, a.out,
                                 cube0, ncub, lds, tinfo);
}

template <typename T, int D, int VW>
__global__ void __launch_bounds__(kThreads) k_batched(const BatchArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int32_t tinfo[2 * kMaxDF];
  T* lds = reinterpret_cast<T*>(smem);
  for (int64_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
    const BatchItem item = a.items[it];
    const Geom g = a.blocks[item.block].g;
    const T* src = a.in[item.block];
    T* dst = a.out[item.block];
    run_item<T, D, VW, false, true>(g, a.orbits + item.orbit, a.reps, a.mats, 1, src, dst,
                                    item.cube0, item.ncubes, lds, tinfo);
    __syncthreads();
  }
}

// Plain copy with the same 16-byte loads and non-temporal stores: the
// achievable HBM ceiling for a read-once / write-once kernel.
__global__ void __launch_bounds__(kThreads) k_copy(const double* __restrict__ in,
                                                   double* __restrict__ out, int64_t nvec) {
  typedef double V __attribute__((ext_vector_type(2)));
  const V* src = reinterpret_cast<const V*>(in);
  V* dst = reinterpret_cast<V*>(out);
  int64_t i0 = (int64_t)blockIdx.x * (kUnroll * kThreads) + threadIdx.x;
  V buf[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    int64_t i = i0 + u * kThreads;
    if (i < nvec) buf[u] = src[i];
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    int64_t i = i0 + u * kThreads;
    if (i < nvec) __builtin_nontemporal_store(buf[u], dst + i);
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

template <typename T, int D>
const void* exec_kernel_d(int vw, bool chain, bool nts) {
  if (chain) return nts ? exec_kernel<T, D, true, true>(vw) : exec_kernel<T, D, true, false>(vw);
  return nts ? exec_kernel<T, D, false, true>(vw) : exec_kernel<T, D, false, false>(vw);
}

template <typename T, int D>
const void* batched_kernel(int vw) {
  if constexpr (sizeof(T) == 8) {
    if (vw == 2) return (const void*)k_batched<T, D, 2>;
    return (const void*)k_batched<T, D, 1>;
  } else {
    if (vw == 4) return (const void*)k_batched<T, D, 4>;
    if (vw == 2) return (const void*)k_batched<T, D, 2>;
    return (const void*)k_batched<T, D, 1>;
  }
}

template <typename T>
const void* pick_exec(int d, int vw, bool chain, bool nts) {
  switch (d) {
    case 2: return exec_kernel_d<T, 2>(vw, chain, nts);
    case 3: return exec_kernel_d<T, 3>(vw, chain, nts);
    default: return exec_kernel_d<T, 4>(vw, chain, nts);
  }
}

template <typename T>
const void* pick_batched(int d, int vw) {
  switch (d) {
    case 2: return batched_kernel<T, 2>(vw);
    case 3: return batched_kernel<T, 3>(vw);
    default: return batched_kernel<T, 4>(vw);
  }
}

template <typename T>
spinsum_status launch_exec(spinsum_plan_s* P, const void* in, void* out, hipStream_t stream,
                           bool adjoint) {
  const Tiling& Tl = P->T;
  if (Tl.nitems <= 0) return SPINSUM_OK;
  const int df = P->G.df;
  const int K = (int)P->stage_a.size();
  const bool chain = (P->flags & SPINSUM_FLAG_CHAIN_STAGES) != 0;
  const T* mats = reinterpret_cast<const T*>(P->d_mats);
  ExecArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.in = reinterpret_cast<const T*>(in);
  a.out = reinterpret_cast<T*>(out);
  a.orbits = reinterpret_cast<const OrbitDev*>(P->d_orbits);
  a.reps = reinterpret_cast<const uint32_t*>(P->d_reps);
  if (!chain) {
    a.mats = mats + (adjoint ? (size_t)df * df : 0);
    a.nmats = 1;
  } else {
    a.mats = mats + 2 * (size_t)df * df + (adjoint ? (size_t)K * df * df : 0);
    a.nmats = K;
  }
  a.g = Tl.g;
  a.nitems = Tl.nitems;
  a.reverse = (P->flags & SPINSUM_FLAG_REVERSE_ORDER) ? 1 : 0;
  a.nt = (P->flags & SPINSUM_FLAG_NO_NT_STORES) ? 0 : 1;
  int64_t grid;
  if (P->flags & SPINSUM_FLAG_NO_XCD_REMAP) {
    a.xcd_per = 0;
    grid = Tl.nitems;
  } else {
    a.xcd_per = (Tl.nitems + 7) / 8;
    grid = a.xcd_per * 8;
  }
  const void* k = pick_exec<T>(P->d, Tl.vw, chain, a.nt != 0);
  size_t shmem = (size_t)Tl.lds_elems * sizeof(T);
  void* kargs[] = {&a};
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) {
      P->last_hip_error = (int)e;
      (void)hipGetLastError();
      return SPINSUM_ERR_HIP;
    }
  }
  hipError_t e = hipLaunchKernel(k, dim3((unsigned)grid), dim3(kThreads), kargs, shmem, stream);
  if (e != hipSuccess) {
    P->last_hip_error = (int)e;
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
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
  a.orbits = reinterpret_cast<const OrbitDev*>(P->d_orbits);
  a.reps = reinterpret_cast<const uint32_t*>(P->d_reps);
  a.mats = reinterpret_cast<const T*>(P->d_mats);
  a.blocks = reinterpret_cast<const BatchBlock*>(P->d_blocks);
  a.items = reinterpret_cast<const BatchItem*>(P->d_items);
  a.nitems = (int64_t)P->items.size();
  a.nt = (P->flags & SPINSUM_FLAG_NO_NT_STORES) ? 0 : 1;
  const void* k = pick_batched<T>(P->d, P->batch_vw);
  size_t shmem = (size_t)P->batch_lds_elems * sizeof(T);
  void* kargs[] = {&a};
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) {
      P->last_hip_error = (int)e;
      (void)hipGetLastError();
      return SPINSUM_ERR_HIP;
    }
  }
  hipError_t e =
      hipLaunchKernel(k, dim3((unsigned)P->batch_grid), dim3(kThreads), kargs, shmem, stream);
  if (e != hipSuccess) {
    P->last_hip_error = (int)e;
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
  return SPINSUM_OK;
}

spinsum_status check_device(spinsum_plan_s* P) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    P->last_hip_error = (int)e;
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
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
}  // namespace spinsum

using namespace spinsum;

extern "C" spinsum_status spinsum_exec(spinsum_plan_t P, const void* in, void* out, void* stream) {
  spinsum_status st = check_tensor_args(P, in, out);
  if (st != SPINSUM_OK || P->elems == 0) return st;
  if (P->dtype == SPINSUM_F32)
    return launch_exec<float>(P, in, out, (hipStream_t)stream, false);
  return launch_exec<double>(P, in, out, (hipStream_t)stream, false);
}

extern "C" spinsum_status spinsum_adjoint(spinsum_plan_t P, const void* grad_out, void* grad_in,
                                          void* stream) {
  spinsum_status st = check_tensor_args(P, grad_out, grad_in);
  if (st != SPINSUM_OK || P->elems == 0) return st;
  if (P->dtype == SPINSUM_F32)
    return launch_exec<float>(P, grad_out, grad_in, (hipStream_t)stream, true);
  return launch_exec<double>(P, grad_out, grad_in, (hipStream_t)stream, true);
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
  if (e != hipSuccess) {
    P->last_hip_error = (int)e;
    (void)hipGetLastError();
    return SPINSUM_ERR_HIP;
  }
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
  const int64_t per = (int64_t)kUnroll * kThreads;
  const int64_t grid = (nvec + per - 1) / per;
  if (grid >= (1ll << 31)) return SPINSUM_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(kThreads), 0, (hipStream_t)stream,
                     (const double*)in, (double*)out, nvec);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPINSUM_OK : SPINSUM_ERR_HIP;
}
