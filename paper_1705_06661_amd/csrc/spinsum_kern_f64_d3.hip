// spinsum_kern_f64_d3.hip -- instantiates the double kernels of libspinsum for
// a group of 3 indices (kernel templates in spinsum_device.h).
#include "spinsum_device.h"

namespace spinsum {

const void* pick_f64_d3(int kind, int vw, bool chain, bool nts, int maxc) {
  return pick_d<double, 3>(kind, vw, chain, nts, maxc);
}

const void* pick_batched_f64_d3(int vw, bool persist) { return batched_kernel<double, 3>(vw, persist); }

const void* pick_cgrad_f64_d3(bool split) { return cgrad_kernel<double, 3>(split); }

const void* pick_pack_f64_d3(bool pack, bool nts, bool persist) {
  return pack_kernel<double, 3>(pack, nts, persist);
}

}  // namespace spinsum
