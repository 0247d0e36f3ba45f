// Kernels of the Bluestein steps (lengths that are not powers of two).
#include "bluestein.h"

namespace dft3d {
void register_kernels_bluestein(std::vector<KernelInfo>& v) {
  const LaunchFn fns[3] = {&launch_bluestein_pad, &launch_bluestein_filter,
                           &launch_bluestein_crop};
  const int lds[3] = {0, 0, 32 * 33 * 8};
  for (int kind = 1; kind <= 3; ++kind) {
    KernelInfo k{0, 0, MODE_ROW, kind == 3 ? MODE_COL : MODE_ROW, 0, kBluesteinThreads,
                 lds[kind - 1], fns[kind - 1], 0, 0, 0};
    k.bluestein = kind;
    v.push_back(k);
  }
}
}  // namespace dft3d
