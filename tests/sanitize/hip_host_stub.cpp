// hip_host_stub.cpp -- the few HIP runtime calls the planner makes, served
// from host memory, for a CPU build of the planner under AddressSanitizer
// and UndefinedBehaviorSanitizer (test infrastructure, not part of the
// library).  "Device" allocations are malloc'd blocks; stub_fail_alloc_at(k)
// makes the k-th allocation after the call fail as out of memory, so every
// clean-up path of plan creation and re-tiling can be driven from a test;
// stub_live_allocations() counts the blocks not yet freed.  The kernels are
// not built here: exec entry points report that no device is present.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <set>

#include "spinsum_plan_host.h"

namespace {
std::set<void*> g_live;
long g_count = 0;
long g_fail_at = 0;
hipError_t g_last = hipSuccess;
}  // namespace

extern "C" void stub_fail_alloc_at(long k) {
  g_fail_at = k;
  g_count = 0;
}
extern "C" long stub_live_allocations(void) { return (long)g_live.size(); }
extern "C" long stub_allocations_made(void) { return g_count; }

extern "C" hipError_t hipMalloc(void** ptr, size_t size) {
  ++g_count;
  if (g_fail_at > 0 && g_count == g_fail_at) {
    *ptr = nullptr;
    g_last = hipErrorOutOfMemory;
    return hipErrorOutOfMemory;
  }
  void* p = std::malloc(size ? size : 1);
  if (!p) return hipErrorOutOfMemory;
  g_live.insert(p);
  *ptr = p;
  return hipSuccess;
}

extern "C" hipError_t hipFree(void* ptr) {
  if (!ptr) return hipSuccess;
  if (g_live.erase(ptr) != 1) std::abort();  // not ours, or freed twice
  std::free(ptr);
  return hipSuccess;
}

extern "C" hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}

extern "C" hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}

extern "C" hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t attr, int) {
  if (attr == hipDeviceAttributeMultiprocessorCount) {
    *v = 256;
  } else if (attr == hipDeviceAttributeMaxSharedMemoryPerBlock) {
    *v = 160 * 1024;
  } else {
    *v = 0;
  }
  return hipSuccess;
}

extern "C" hipError_t hipGetLastError(void) {
  hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}

extern "C" hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* prop, int) {
  std::memset(prop, 0, sizeof(*prop));
  std::strcpy(prop->gcnArchName, "gfx950");
  std::strcpy(prop->name, "host stub");
  prop->multiProcessorCount = 256;
  return hipSuccess;
}

extern "C" hipError_t hipEventCreate(hipEvent_t*) { return hipErrorNotSupported; }
extern "C" hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
extern "C" hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipErrorNotSupported; }
extern "C" hipError_t hipEventSynchronize(hipEvent_t) { return hipErrorNotSupported; }
extern "C" hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t) {
  return hipErrorNotSupported;
}

namespace spinsum {
spinsum_status cache_occupancy(spinsum_plan_s* P) {
  P->occ_blocks = 2;
  return SPINSUM_OK;
}
}  // namespace spinsum

extern "C" spinsum_status spinsum_exec(spinsum_plan_t, const void*, void*, void*) {
  return SPINSUM_ERR_NO_DEVICE;
}
extern "C" spinsum_status spinsum_exec_batched(spinsum_plan_t, const void* const*, void* const*,
                                               void*) {
  return SPINSUM_ERR_NO_DEVICE;
}
