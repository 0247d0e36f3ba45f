// Rader pass kernels (prime lengths n with n - 1 free of prime factors
// above 13), per tile shape (T pencils of up to NMAX points, n + 1 <= NMAX,
// T * NMAX = 8192) and variant (as the mixed-radix kernels: 2 runs the
// radix-11 and radix-13 stages).
#include "rader.h"

namespace dft3d {
void register_kernels_rader(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_rader<256, 32, 512, 1>());
  v.push_back(kernel_info_rader<64, 128, 512, 1>());
  v.push_back(kernel_info_rader<16, 512, 512, 1>());
  v.push_back(kernel_info_rader<8, 1024, 512, 1>());
  v.push_back(kernel_info_rader<4, 2048, 512, 1>());
  v.push_back(kernel_info_rader<2, 4096, 512, 1>());
  v.push_back(kernel_info_rader<256, 32, 256, 2>());
  v.push_back(kernel_info_rader<64, 128, 256, 2>());
  v.push_back(kernel_info_rader<16, 512, 256, 2>());
  v.push_back(kernel_info_rader<8, 1024, 256, 2>());
  v.push_back(kernel_info_rader<4, 2048, 256, 2>());
  v.push_back(kernel_info_rader<2, 4096, 256, 2>());
}
}  // namespace dft3d
