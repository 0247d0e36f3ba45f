// Fused volumetric two-axis kernels for split factors 16 and 32, natural and
// shuffled layouts, and the inverse from the shuffled layout.
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
  // shuffled layout: the fused axis's output left in digit order; runs
  // contiguous at a = 32 in tiles of 8 runs first (68 KB of LDS, two
  // workgroups per CU; the shuffled stores stay contiguous along l':
  // 1024^3 forward 14.43 -> 13.97 ms)
  v.push_back(kernel_info_fused_axes<32, 8, 1, 0, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 1, 0, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 0, 1>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 0, 1>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 0, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 1, 1, 1>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 1, 1>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 1, 1>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 1, 1>());
  // inverse from the shuffled layout: the transposed pass, in place (the
  // same 8-run tiles first: 1024^3 14.73 -> 14.17 ms)
  v.push_back(kernel_info_fused_axes<32, 8, 1, 0, 3>());
  v.push_back(kernel_info_fused_axes<32, 16, 1, 0, 3>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 0, 3>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 0, 3>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 0, 3>());
  v.push_back(kernel_info_fused_axes<32, 16, 1, 1, 3>());
  v.push_back(kernel_info_fused_axes<32, 16, 0, 1, 3>());
  v.push_back(kernel_info_fused_axes<16, 16, 1, 1, 3>());
  v.push_back(kernel_info_fused_axes<16, 32, 0, 1, 3>());
}
}  // namespace dft3d
