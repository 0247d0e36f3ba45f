// One-pass Bluestein axis kernels (lengths that are not powers of two), one
// per convolution length m = 8 .. 8192 and tile.
#include "bluestein.h"

namespace dft3d {
void register_kernels_bluestein(std::vector<KernelInfo>& v) {
  // The first tile of each length is its default.  Measured on MI355X
  // (250^3 .. 2000^2 x 256): smaller tiles, or 16 elements per thread with
  // twice the waves per SIMD, do not run faster except at m = 512, where
  // four pencils per workgroup beat sixteen by 10%; the kernel is bound by
  // its arithmetic and memory-instruction issue, not by occupancy.
  v.push_back(kernel_info_bluestein<8, 256>());
  v.push_back(kernel_info_bluestein<16, 256>());
  v.push_back(kernel_info_bluestein<16, 64>());
  v.push_back(kernel_info_bluestein<32, 128>());
  v.push_back(kernel_info_bluestein<32, 32>());
  v.push_back(kernel_info_bluestein<64, 64>());
  v.push_back(kernel_info_bluestein<64, 16>());
  v.push_back(kernel_info_bluestein<128, 32>());
  v.push_back(kernel_info_bluestein<128, 8>());
  v.push_back(kernel_info_bluestein<256, 32>());
  v.push_back(kernel_info_bluestein<256, 8>());
  v.push_back(kernel_info_bluestein<512, 4>());
  v.push_back(kernel_info_bluestein<512, 8>());
  v.push_back(kernel_info_bluestein<512, 16>());
  v.push_back(kernel_info_bluestein<1024, 16>());
  v.push_back(kernel_info_bluestein<1024, 8>());
  v.push_back(kernel_info_bluestein<1024, 4>());
  v.push_back(kernel_info_bluestein<2048, 8>());
  v.push_back(kernel_info_bluestein<2048, 4>());
  v.push_back(kernel_info_bluestein<2048, 2>());
  v.push_back(kernel_info_bluestein<4096, 4>());
  v.push_back(kernel_info_bluestein<4096, 2>());
  v.push_back(kernel_info_bluestein<4096, 1>());
  v.push_back(kernel_info_bluestein<8192, 2>());
  v.push_back(kernel_info_bluestein<8192, 1>());
}
}  // namespace dft3d
