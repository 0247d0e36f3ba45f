// Rader pass kernels compiled for one prime each (the prime and the radix
// code of n - 1 as the planner packs it as compile-time constants; a
// kernel whose code differs is never picked).  Primes spread over the
// supported range; the others take the Bluestein pass by default.
// Measured on MI355X, pencil plans, Rader / Bluestein time: 197^3 0.16 /
// 0.25 ms, 257^3 0.41 / 0.85, 641^3 4.8 / 12.3, 1009^3 19.2 / 37.7,
// 2017 x 2017 x 64 6.8 / 9.5; at 127^3 Rader was slower (0.087 / 0.051 ms),
// so no kernel is compiled below 197.
#include "rader.h"

namespace dft3d {
void register_kernels_rader_fixed(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_rader_fixed<32, 256, 512, 197, 0x40707>());  // 196 = 7*7*4
  v.push_back(kernel_info_rader_fixed<16, 512, 512, 257, 0x1010>());  // 256 = 16*16
  v.push_back(kernel_info_rader_fixed<16, 512, 512, 281, 0x40a07>());  // 280 = 7*10*4
  v.push_back(kernel_info_rader_fixed<16, 512, 512, 401, 0x40a0a>());  // 400 = 10*10*4
  v.push_back(kernel_info_rader_fixed<8, 1024, 512, 577, 0x8080303>());  // 576 = 3*3*8*8
  v.push_back(kernel_info_rader_fixed<8, 1024, 512, 641, 0x8080a>());  // 640 = 10*8*8
  v.push_back(kernel_info_rader_fixed<8, 1024, 512, 769, 0x101003>());  // 768 = 3*16*16
  v.push_back(kernel_info_rader_fixed<8, 1024, 512, 1009, 0x10030307>());  // 1008 = 7*3*3*16
  v.push_back(kernel_info_rader_fixed<4, 2048, 512, 1201, 0x40a0a03>());  // 1200 = 3*10*10*4
  v.push_back(kernel_info_rader_fixed<4, 2048, 512, 1601, 0x100a0a>());  // 1600 = 10*10*16
  v.push_back(kernel_info_rader_fixed<4, 2048, 512, 2017, 0x804030307>());  // 2016 = 7*3*3*4*8
  v.push_back(kernel_info_rader_fixed<2, 4096, 512, 2593, 0x80403030303>());  // 2592 = 3*3*3*3*4*8
  v.push_back(kernel_info_rader_fixed<2, 4096, 512, 3001, 0x803050505>());  // 3000 = 5*5*5*3*8
  v.push_back(kernel_info_rader_fixed<2, 4096, 512, 4001, 0x804050505>());  // 4000 = 5*5*5*4*8
}
}  // namespace dft3d
