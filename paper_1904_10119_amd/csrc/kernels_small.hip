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
}
}  // namespace dft3d
