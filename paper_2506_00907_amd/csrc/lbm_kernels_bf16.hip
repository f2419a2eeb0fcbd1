// Kernel instantiations for BF16 population storage.
#include "lbm_device.hpp"

namespace lbmi {
KernelSet kernels_bf16(int fl, int sl, int ml, int nc, int ns) { return select_kernels<BF16S>(fl, sl, ml, nc, ns); }
}  // namespace lbmi
