// Split-precision MFMA pass kernels for lengths 128..512.
#include "mfma_kernel.h"

namespace dft3d {
void register_kernels_mfma_b(std::vector<KernelInfo>& v) {
  add_mfma_kernels<128>(v);
  add_mfma_kernels<256>(v);
  add_mfma_kernels<512>(v);
}
}  // namespace dft3d
