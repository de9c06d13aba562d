// spinsum_kern_f32_d3.hip -- instantiates the float kernels of libspinsum for
// a group of 3 indices (kernel templates in spinsum_device.h).
#include "spinsum_device.h"

namespace spinsum {

const void* pick_f32_d3(int kind, int vw, bool chain, bool nts, int maxc) {
  return pick_d<float, 3>(kind, vw, chain, nts, maxc);
}

const void* pick_batched_f32_d3(int vw, bool persist) { return batched_kernel<float, 3>(vw, persist); }

const void* pick_cgrad_f32_d3(bool split) { return cgrad_kernel<float, 3>(split); }

const void* pick_pack_f32_d3(bool pack, bool nts, bool persist) {
  return pack_kernel<float, 3>(pack, nts, persist);
}

}  // namespace spinsum
