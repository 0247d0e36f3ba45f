// The passes as two half-length transforms (halves_kernel.h): length 2048
// rotated on write and strided in place (16 pencils), length 1024 strided in
// place (32 pencils); persistent forms for the first and the last (the
// strided 2048 pass measured slower in its persistent form and has none).
// The 1024-point rotate-on-write pass in 32-pencil
// halves measured slower than the persistent 16-pencil kernel (3.8 against
// 3.5 ms at 1024^3) and is not compiled.
#include "halves_kernel.h"

namespace dft3d {
void register_kernels_halves(std::vector<KernelInfo>& v) {
  add_halves_kernels<2048, 16, MODE_ROW, MODE_COL, true>(v);
  add_halves_kernels<2048, 16, MODE_COL, MODE_COL, false>(v);
  add_halves_kernels<1024, 32, MODE_COL, MODE_COL, true>(v);
}
}  // namespace dft3d
