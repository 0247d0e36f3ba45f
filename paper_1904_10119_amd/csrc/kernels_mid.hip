// Pass kernels for transform lengths 128..512.
#include "pass_kernel.h"

namespace dft3d {
void register_kernels_mid(std::vector<KernelInfo>& v) {
  add_kernels<128, 16>(v);
  add_kernels<128, 32>(v);
  add_kernels<128, 64>(v);
  add_kernels<256, 16>(v);
  add_kernels<256, 32>(v);
  add_kernels<512, 8>(v);
  add_kernels<512, 16>(v);
  add_kernels<512, 32>(v);
  add_persistent_kernels<512, 16, Blocking<512>>(v);
  add_persistent_kernels<512, 32, Blocking<512>>(v);
}
}  // namespace dft3d
