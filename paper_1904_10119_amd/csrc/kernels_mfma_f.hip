// Split-precision MFMA rotate-on-write passes of length 2048 in the wide
// one-tile form: 8 pencils per workgroup (1024 threads, one workgroup per
// CU) where the default tile has 4, so the rotated store writes 64-byte
// row segments instead of 32 (2048 x 1024 x 512 bf16x6: 7.84 -> 6.23 ms per
// launch).  At length 1024 the wide form (16 pencils, 128-byte segments,
// byte counters 1.00 x instead of 1.24 x) measured slower than two
// workgroups of 8 pencils per CU (5.38 against 4.83 ms) and is not compiled.
#include "mfma_kernel.h"

namespace dft3d {
void register_kernels_mfma_f(std::vector<KernelInfo>& v) {
  add_mfma_wide_kernels<2048, 32>(v);
  add_mfma_wide_kernels<2048, 16>(v);
}
}  // namespace dft3d
