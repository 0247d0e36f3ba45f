// Fused volumetric two-axis kernels for split factors 16 and 32, natural and
// shuffled layouts.
#include "fused_axes_kernel.h"

namespace dft3d {
void register_kernels_fused(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_fused_axes<32, 16, 1, 0>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 0>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 0>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 0>());
  v.push_back(kernel_info_fused_axes<32, 16, 1, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 1>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 1>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 1>());
  // shuffled layout: the fused axis's output left in digit order
  v.push_back(kernel_info_fused_axes<32, 16, 1, 0, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 0, 1>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 0, 1>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 0, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 1, 1, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 1, 1>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 1, 1>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 1, 1>());
}
}  // namespace dft3d
