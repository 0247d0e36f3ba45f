// Twiddle tables: the only FP64 step of the library.
//
// w_n^m = exp(-2 pi i m / n) (eq. (4) entries, forward direction).  The
// exponent is reduced exactly in integers to a whole number of quarter turns
// plus an angle in [0, pi/2); that angle is folded into [0, pi/4] so the C
// library's cos and sin are called only on small arguments, and 0, +-1 and
// +-sqrt(1/2) are exact.  Each entry is rounded once to FP32.
#include <cmath>

#include "internal.h"

namespace dft3d {

void make_roots(int64_t n, float2* out) {
  const double half_pi = 1.57079632679489661923132169163975144;
  for (int64_t m = 0; m < n; ++m) {
    const int64_t q = (4 * m) / n;      // quarter turns
    const int64_t rem = 4 * m - q * n;  // (pi/2) * rem / n left over
    double c, s;
    if (rem == 0) {
      c = 1.0; s = 0.0;
    } else if (2 * rem == n) {
      c = std::sqrt(0.5); s = c;
    } else if (2 * rem < n) {
      const double x = half_pi * (double)rem / (double)n;
      c = std::cos(x); s = std::sin(x);
    } else {
      const double x = half_pi * (double)(n - rem) / (double)n;
      c = std::sin(x); s = std::cos(x);
    }
    for (int64_t k = 0; k < q; ++k) {  // times i per quarter turn
      const double t = c;
      c = -s;
      s = t;
    }
    out[m] = make_float2((float)c, (float)(-s));
  }
}

}  // namespace dft3d
