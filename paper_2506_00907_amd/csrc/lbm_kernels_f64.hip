// Kernel instantiations for F64 population storage.
#include "lbm_device.hpp"

namespace lbmi {
KernelSet kernels_f64(int fl, int sl, int ml, int nc, int ns) { return select_kernels<F64S>(fl, sl, ml, nc, ns); }
}  // namespace lbmi
