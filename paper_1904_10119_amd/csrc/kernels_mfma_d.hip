// Split-precision MFMA pass kernels with length-32 leaves, lengths 32..256.
#include "mfma_kernel.h"

namespace dft3d {
void register_kernels_mfma_d(std::vector<KernelInfo>& v) {
  add_mfma_kernels<32, 32>(v);
  add_mfma_kernels<64, 32>(v);
  add_mfma_kernels<128, 32>(v);
  add_mfma_kernels<256, 32>(v);
}
}  // namespace dft3d
