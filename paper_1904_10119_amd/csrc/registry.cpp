// Registry of the compiled pass kernels.
#include "internal.h"

namespace dft3d {

void register_kernels_small(std::vector<KernelInfo>& v);
void register_kernels_mid(std::vector<KernelInfo>& v);
void register_kernels_1k(std::vector<KernelInfo>& v);
void register_kernels_big(std::vector<KernelInfo>& v);

const std::vector<KernelInfo>& kernel_registry() {
  static const std::vector<KernelInfo> table = [] {
    std::vector<KernelInfo> v;
    register_kernels_small(v);
    register_kernels_mid(v);
    register_kernels_1k(v);
    register_kernels_big(v);
    return v;
  }();
  return table;
}

const KernelInfo* find_kernel(int n, int tile, int lmode, int smode, int post_twiddle) {
  for (const KernelInfo& k : kernel_registry())
    if (k.n == n && k.tile == tile && k.lmode == lmode && k.smode == smode &&
        k.post_twiddle == post_twiddle)
      return &k;
  return nullptr;
}

}  // namespace dft3d
