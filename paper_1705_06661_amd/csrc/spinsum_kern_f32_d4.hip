// spinsum_kern_f32_d4.hip -- instantiates the float kernels of libspinsum for
// a group of 4 indices (kernel templates in spinsum_device.h).
#include "spinsum_device.h"

namespace spinsum {

const void* pick_f32_d4(int kind, int vw, bool chain, bool nts, int maxc) {
  return pick_d<float, 4>(kind, vw, chain, nts, maxc);
}

const void* pick_batched_f32_d4(int vw, bool persist) { return batched_kernel<float, 4>(vw, persist); }

const void* pick_cgrad_f32_d4(bool split) { return cgrad_kernel<float, 4>(split); }

const void* pick_pack_f32_d4(bool pack, bool nts, bool persist) {
  return pack_kernel<float, 4>(pack, nts, persist);
}

}  // namespace spinsum
