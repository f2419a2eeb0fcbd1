// Kernel instantiations for BF16 population storage.
#include "lbm_device.hpp"

namespace lbmi {
KernelSet kernels_bf16(int fl, int sl, int ml, int nc) { return select_kernels<BF16S>(fl, sl, ml, nc); }
}  // namespace lbmi
