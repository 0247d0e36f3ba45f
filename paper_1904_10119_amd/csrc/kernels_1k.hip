// Pass kernels for transform length 1024.
#include "pass_kernel.h"

namespace dft3d {
void register_kernels_1k(std::vector<KernelInfo>& v) {
  add_kernels<1024, 8>(v);
  add_kernels<1024, 16>(v);
  add_persistent_kernels<1024, 16, Blocking<1024>>(v);
  add_group_kernels<1024, 16, Blocking<1024>>(v);
}
}  // namespace dft3d
