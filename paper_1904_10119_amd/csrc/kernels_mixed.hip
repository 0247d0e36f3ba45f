// Mixed-radix pencil pass kernels (lengths whose prime factors are at most
// 13), per tile shape (T pencils of up to NMAX points, T * NMAX = 8192) and
// variant: 1 for lengths without the factors 11 and 13 (512 threads), 2
// with them (256 threads: its registers leave room for two workgroups per
// CU); each as the rotating pass (ROW load, COL store) and the two
// in-layout passes (ROW -> ROW, COL -> COL) of the slab and volumetric
// schedules.
#include "mixed_kernel.h"

namespace dft3d {
void register_kernels_mixed(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_mixed<256, 32, 512, 1>());
  v.push_back(kernel_info_mixed<256, 32, 512, 1, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<256, 32, 512, 1, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<64, 128, 512, 1>());
  v.push_back(kernel_info_mixed<64, 128, 512, 1, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<64, 128, 512, 1, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<16, 512, 512, 1>());
  v.push_back(kernel_info_mixed<16, 512, 512, 1, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<16, 512, 512, 1, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<8, 1024, 512, 1>());
  v.push_back(kernel_info_mixed<8, 1024, 512, 1, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<8, 1024, 512, 1, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<4, 2048, 512, 1>());
  v.push_back(kernel_info_mixed<4, 2048, 512, 1, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<4, 2048, 512, 1, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<2, 4096, 512, 1>());
  v.push_back(kernel_info_mixed<2, 4096, 512, 1, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<2, 4096, 512, 1, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<256, 32, 256, 2>());
  v.push_back(kernel_info_mixed<256, 32, 256, 2, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<256, 32, 256, 2, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<64, 128, 256, 2>());
  v.push_back(kernel_info_mixed<64, 128, 256, 2, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<64, 128, 256, 2, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<16, 512, 256, 2>());
  v.push_back(kernel_info_mixed<16, 512, 256, 2, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<16, 512, 256, 2, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<8, 1024, 256, 2>());
  v.push_back(kernel_info_mixed<8, 1024, 256, 2, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<8, 1024, 256, 2, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<4, 2048, 256, 2>());
  v.push_back(kernel_info_mixed<4, 2048, 256, 2, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<4, 2048, 256, 2, MODE_COL, MODE_COL>());
  v.push_back(kernel_info_mixed<2, 4096, 256, 2>());
  v.push_back(kernel_info_mixed<2, 4096, 256, 2, MODE_ROW, MODE_ROW>());
  v.push_back(kernel_info_mixed<2, 4096, 256, 2, MODE_COL, MODE_COL>());
}
}  // namespace dft3d
