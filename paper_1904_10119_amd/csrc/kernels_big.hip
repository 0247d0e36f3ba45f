// Pass kernels for transform lengths 2048 and 4096.
#include "pass_kernel.h"

namespace dft3d {
void register_kernels_big(std::vector<KernelInfo>& v) {
  add_kernels<2048, 4>(v);
  add_kernels<2048, 8>(v);
  add_persistent_kernels<2048, 8, BlockingWide<2048>>(v);
  add_kernels<4096, 2>(v);
  add_kernels<4096, 4>(v);
}
}  // namespace dft3d
