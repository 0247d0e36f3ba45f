// Pass kernels for transform lengths 1..64.
#include "pass_kernel.h"

namespace dft3d {
void register_kernels_small(std::vector<KernelInfo>& v) {
  add_kernels<1, 256>(v);
  add_kernels<2, 256>(v);
  add_kernels<4, 256>(v);
  add_kernels<8, 64>(v);
  add_kernels<8, 256>(v);
  add_kernels<16, 64>(v);
  add_kernels<16, 256>(v);
  add_kernels<32, 64>(v);
  add_kernels<32, 128>(v);
  add_kernels<64, 16>(v);
  add_kernels<64, 32>(v);
  add_kernels<64, 64>(v);
  add_row_twiddle_kernels<2, 256>(v);
  add_row_twiddle_kernels<4, 256>(v);
  add_row_twiddle_kernels<8, 256>(v);
  add_row_twiddle_kernels<16, 256>(v);
  add_row_twiddle_kernels<32, 128>(v);
  add_row_twiddle_kernels<64, 64>(v);
  // plain copies of a pass's points (move-only option, copy mode)
  v.push_back(kernel_info_copy<1>());
  v.push_back(kernel_info_copy<2>());
  v.push_back(kernel_info_copy<4>());
  v.push_back(kernel_info_copy<8>());
  v.push_back(kernel_info_copy<16>());
  v.push_back(kernel_info_copy<32>());
  v.push_back(kernel_info_copy<64>());
  v.push_back(kernel_info_copy<128>());
  v.push_back(kernel_info_copy<256>());
  v.push_back(kernel_info_copy<512>());
  v.push_back(kernel_info_copy<1024>());
  v.push_back(kernel_info_copy<2048>());
  v.push_back(kernel_info_copy<4096>());
}
}  // namespace dft3d
