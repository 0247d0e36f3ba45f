// Split-precision MFMA pass kernels for lengths 1024..4096.
#include "mfma_kernel.h"

namespace dft3d {
void register_kernels_mfma_c(std::vector<KernelInfo>& v) {
  add_mfma_kernels<1024>(v);
  add_mfma_kernels<2048>(v);
  add_mfma_kernels<4096>(v);
}
}  // namespace dft3d
