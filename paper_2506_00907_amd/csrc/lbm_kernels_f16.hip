// Kernel instantiations for F16 population storage.
#include "lbm_device.hpp"

namespace lbmi {
KernelSet kernels_f16(int fl, int sl, int ml, int nc, int ns) { return select_kernels<F16S>(fl, sl, ml, nc, ns); }
}  // namespace lbmi
