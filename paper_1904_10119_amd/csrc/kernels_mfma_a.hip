// Split-precision MFMA pass kernels for lengths 16..64.
#include "mfma_kernel.h"

namespace dft3d {
void register_kernels_mfma_a(std::vector<KernelInfo>& v) {
  add_mfma_kernels<16>(v);
  add_mfma_kernels<32>(v);
  add_mfma_kernels<64>(v);
}
}  // namespace dft3d
