// Pencil index decomposition with fields of any count, for the passes of
// lengths other than powers of two (mixed-radix and Bluestein kernels).
//
// PassArgs normally splits pencil b into bit fields (pencil_offset in
// pass_kernel.h).  When a field other than the last has a count that is not
// a power of two (a slab or volumetric pass over a shape with such an
// axis), the planner sets s0 = -1 and m0, m1 to the counts of the first two
// fields; the fields are then b0 = b mod m0, b1 = (b div m0) mod m1,
// b2 = b div (m0 m1).  The divisions run once per pencil of a tile.
#pragma once

#include "pass_kernel.h"

namespace dft3d {

__device__ __forceinline__ int64_t pencil_offset_any(int64_t b, int64_t m0, int64_t m1,
                                                     int s0, int s1, int64_t st0,
                                                     int64_t st1, int64_t st2) {
  if (s0 >= 0) return pencil_offset(b, m0, m1, s0, s1, st0, st1, st2);
  int64_t b0, b1, b2;
  if (b < (int64_t(1) << 32) && m0 < (int64_t(1) << 32) && m1 < (int64_t(1) << 32)) {
    const uint32_t u = (uint32_t)b, c0 = (uint32_t)m0, c1 = (uint32_t)m1;
    const uint32_t q = u / c0, r = q / c1;
    b0 = u - q * c0;
    b1 = q - r * c1;
    b2 = r;
  } else {
    const uint64_t q = (uint64_t)b / (uint64_t)m0, r = q / (uint64_t)m1;
    b0 = (int64_t)((uint64_t)b - q * (uint64_t)m0);
    b1 = (int64_t)(q - r * (uint64_t)m1);
    b2 = (int64_t)r;
  }
  return b2 * st2 + b1 * st1 + b0 * st0;
}

}  // namespace dft3d
