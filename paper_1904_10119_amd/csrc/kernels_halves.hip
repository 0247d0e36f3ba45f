// The two-halves rotate-on-write pass of length 2048 (16-pencil tiles):
// ordinary and streaming accesses, and their move-only twins.
#include "halves_kernel.h"

namespace dft3d {
void register_kernels_halves(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_halves<16, 0>());
  v.push_back(kernel_info_halves<16, 1>());
  v.push_back(kernel_info_halves<16, 4>());
  v.push_back(kernel_info_halves<16, 5>());
}
}  // namespace dft3d
