// Mixed-radix pass kernels compiled for one common length each (length and
// radix code as compile-time constants; the code is the one the planner
// packs for the length, a kernel whose code differs is never picked).
#include "mixed_kernel.h"

namespace dft3d {
void register_kernels_mixed_fixed(std::vector<KernelInfo>& v) {
  const size_t first = v.size();
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 48, 0x1003>());  // 3*16
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 60, 0x20A03>());  // 3*10*2
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 72, 0x80303>());  // 3*3*8
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 80, 0x80A>());  // 10*8
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 96, 0x80403>());  // 3*4*8
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 100, 0xA0A>());  // 10*10
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 120, 0x40A03>());  // 3*10*4
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 125, 0x50505>());  // 5*5*5
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 144, 0x100303>());  // 3*3*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 160, 0x100A>());  // 10*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 192, 0x80803>());  // 3*8*8
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 200, 0x20A0A>());  // 10*10*2
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 240, 0x80A03>());  // 3*10*8
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 250, 0xA0505>());  // 5*5*10
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 300, 0xA0A03>());  // 3*10*10
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 320, 0x8040A>());  // 10*4*8
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 384, 0x100803>());  // 3*8*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 400, 0x40A0A>());  // 10*10*4
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 480, 0x100A03>());  // 3*10*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 500, 0xA0A05>());  // 5*10*10
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 600, 0x20A0A03>());  // 3*10*10*2
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 640, 0x8080A>());  // 10*8*8
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 768, 0x101003>());  // 3*16*16
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 800, 0x80A0A>());  // 10*10*8
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 960, 0x8040A03>());  // 3*10*4*8
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 1000, 0xA0A0A>());  // 10*10*10
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 1200, 0x40A0A03>());  // 3*10*10*4
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 1536, 0x8080803>());  // 3*8*8*8
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 2000, 0x20A0A0A>());  // 10*10*10*2
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 2400, 0x804030505>());  // 5*5*3*4*8
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 2500, 0x405050505>());  // 5*5*5*5*4
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 3000, 0x803050505>());  // 5*5*5*3*8
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 3072, 0x808040403>());  // 3*4*4*8*8
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 3200, 0x804040505>());  // 5*5*4*4*8
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 3600, 0x40403030505>());  // 5*5*3*3*4*4
  v.push_back(kernel_info_mixed_fixed<2, 4096, 512, 4000, 0x804050505>());  // 5*5*5*4*8
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 56, 0x807>());  // 7*8
  v.push_back(kernel_info_mixed_fixed<64, 128, 512, 112, 0x1007>());  // 7*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 168, 0x80307>());  // 7*3*8
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 224, 0x80407>());  // 7*4*8
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 336, 0x100307>());  // 7*3*16
  v.push_back(kernel_info_mixed_fixed<16, 512, 512, 448, 0x80807>());  // 7*8*8
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 672, 0x8040307>());  // 7*3*4*8
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 896, 0x100807>());  // 7*8*16
  v.push_back(kernel_info_mixed_fixed<8, 1024, 512, 1008, 0x10030307>());  // 7*3*3*16
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 1344, 0x8080307>());  // 7*3*8*8
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 1792, 0x101007>());  // 7*16*16
  v.push_back(kernel_info_mixed_fixed<4, 2048, 512, 2016, 0x804030307>());  // 7*3*3*4*8
  // the same kernels for the in-layout passes (ROW -> ROW, COL -> COL):
  // the pass arguments carry the strides; measured at 1000^3 (slab) they
  // beat the generic in-layout forms (rows 2.85 vs 3.0 ms, columns 5.3 vs
  // 9.3 ms)
  const size_t rotating = v.size();
  for (int m = 0; m < 2; ++m)
    for (size_t i = first; i < rotating; ++i) {
      KernelInfo k = v[i];
      k.lmode = k.smode = m == 0 ? MODE_ROW : MODE_COL;
      v.push_back(k);
    }
}
}  // namespace dft3d
