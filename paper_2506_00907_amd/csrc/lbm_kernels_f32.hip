// Kernel instantiations for F32 population storage.
#include "lbm_device.hpp"

namespace lbmi {
KernelSet kernels_f32(int fl, int sl, int ml, int nc, int ns) { return select_kernels<F32S>(fl, sl, ml, nc, ns); }
}  // namespace lbmi
