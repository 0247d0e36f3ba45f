// Split-precision MFMA pass kernels with length-32 leaves, lengths 1024..4096.
#include "mfma_kernel.h"

namespace dft3d {
void register_kernels_mfma_e(std::vector<KernelInfo>& v) {
  add_mfma_kernels<1024, 32>(v);
  add_mfma_kernels<2048, 32>(v);
  add_mfma_kernels<4096, 32>(v);
}
}  // namespace dft3d
