// Mixed-radix pencil pass kernels (lengths whose prime factors are at most
// 13), per tile shape (T pencils of up to NMAX points, T * NMAX = 8192) and
// variant: 1 for lengths without the factors 11 and 13 (512 threads), 2
// with them (256 threads: its registers leave room for two workgroups per
// CU).
#include "mixed_kernel.h"

namespace dft3d {
void register_kernels_mixed(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_mixed<256, 32, 512, 1>());
  v.push_back(kernel_info_mixed<64, 128, 512, 1>());
  v.push_back(kernel_info_mixed<16, 512, 512, 1>());
  v.push_back(kernel_info_mixed<8, 1024, 512, 1>());
  v.push_back(kernel_info_mixed<4, 2048, 512, 1>());
  v.push_back(kernel_info_mixed<2, 4096, 512, 1>());
  v.push_back(kernel_info_mixed<256, 32, 256, 2>());
  v.push_back(kernel_info_mixed<64, 128, 256, 2>());
  v.push_back(kernel_info_mixed<16, 512, 256, 2>());
  v.push_back(kernel_info_mixed<8, 1024, 256, 2>());
  v.push_back(kernel_info_mixed<4, 2048, 256, 2>());
  v.push_back(kernel_info_mixed<2, 4096, 256, 2>());
  // compiled for one common length each, with the radix code the planner
  // packs for it (a kernel whose code differs is never picked)
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 96, 0x80403>());  // 3*4*8
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 100, 0xA0A>());  // 10*10
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 120, 0x40A03>());  // 3*10*4
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 125, 0x50505>());  // 5*5*5
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 200, 0x20A0A>());  // 10*10*2
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 250, 0xA0505>());  // 5*5*10
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 384, 0x100803>());  // 3*8*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 500, 0xA0A05>());  // 5*10*10
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 768, 0x101003>());  // 3*16*16
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 1000, 0xA0A0A>());  // 10*10*10
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 1536, 0x8080803>());  // 3*8*8*8
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 2000, 0x20A0A0A>());  // 10*10*10*2
}
}  // namespace dft3d
