// Device building blocks for the batched 1D FFT passes: complex arithmetic,
// compile-time roots of unity, and in-register DFTs of length 2..64.
//
// Every DFT here is the forward transform y_k = sum_j x_j w_R^{jk} with
// w_R = exp(-2 pi i / R) (Section 2.1, eqs. (1)-(2)); the inverse is taken
// as conj(DFT(conj(x))) by the pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace dft3d {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// a * (-i)
__device__ __forceinline__ float2 mul_neg_i(float2 a) { return make_float2(a.y, -a.x); }
// a * (+i)
__device__ __forceinline__ float2 mul_pos_i(float2 a) { return make_float2(-a.y, a.x); }

// ---- compile-time roots of unity (FP64, rounded once to FP32) ----
//
// cos and sin of 2 pi m / R are reduced exactly to the first octant with
// integer arithmetic, evaluated there by Taylor series in double precision
// (|x| <= pi/4, 13 terms: truncation far below 1e-17) and restored by
// symmetry, so 0, +-1 and +-sqrt(1/2) come out exact.
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kSqrtHalf = 0.70710678118654752440084436210484904;

constexpr double sin_series(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 13; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 13; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

struct CosSin {
  double c, s;
};

// (cos, sin) of 2 pi m / R.
constexpr CosSin unit_angle(long m, long R) {
  m %= R;
  if (m < 0) m += R;
  const long q = (4 * m) / R;       // whole quarter turns
  const long rem = 4 * m - q * R;   // remainder, in units of (pi/2)/R
  double c = 1.0, s = 0.0;
  if (rem == 0) {
    c = 1.0; s = 0.0;
  } else if (2 * rem == R) {
    c = kSqrtHalf; s = kSqrtHalf;
  } else if (2 * rem < R) {
    const double x = (kPi / 2) * (double)rem / (double)R;
    c = cos_series(x); s = sin_series(x);
  } else {
    const double x = (kPi / 2) * (double)(R - rem) / (double)R;
    c = sin_series(x); s = cos_series(x);
  }
  for (long i = 0; i < q; ++i) {  // multiply by i once per quarter turn
    const double t = c;
    c = -s;
    s = t;
  }
  return CosSin{c, s};
}

// v * w_R^M with w_R = exp(-2 pi i / R); trivial factors become sign flips
// and swaps, the eighth turns a single scale.
template <int M, int R>
__device__ __forceinline__ float2 mul_root(float2 v) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (4 * m == R) {
    return mul_neg_i(v);
  } else if constexpr (2 * m == R) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * m == 3 * R) {
    return mul_pos_i(v);
  } else if constexpr (8 * m == R) {
    constexpr float h = (float)kSqrtHalf;
    return make_float2((v.x + v.y) * h, (v.y - v.x) * h);
  } else if constexpr (8 * m == 3 * R) {
    constexpr float h = (float)kSqrtHalf;
    return make_float2((v.y - v.x) * h, -(v.x + v.y) * h);
  } else if constexpr (8 * m == 5 * R) {
    constexpr float h = (float)kSqrtHalf;
    return make_float2(-(v.x + v.y) * h, (v.x - v.y) * h);
  } else if constexpr (8 * m == 7 * R) {
    constexpr float h = (float)kSqrtHalf;
    return make_float2((v.x - v.y) * h, (v.x + v.y) * h);
  } else {
    constexpr CosSin cs = unit_angle(m, R);
    constexpr float c = (float)cs.c;
    constexpr float s = -(float)cs.s;  // forward root: exp(-i theta)
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// Compile-time loop: f(std::integral_constant<int, 0>) ... f(<N-1>).
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f,
                                                std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// In-register forward DFT of length R (a power of two <= 64), natural order
// in and out.  R > 4 splits R = A * B (x index j = b + B a, output index
// k = a' + A b'): DFT_A over a for every b, twiddle w_R^{b a'}, DFT_B over b
// for every a' -- the four-step identity of eq. (3) applied in registers.
template <int R>
__device__ __forceinline__ void dft(float2* x) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    const float2 b0 = cadd(x[1], x[3]), b1 = mul_neg_i(csub(x[1], x[3]));
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  } else {
    constexpr int A = (R >= 64) ? 8 : (R >= 16 ? 4 : 2);
    constexpr int B = R / A;
    float2 z[R];
    static_for<B>([&](auto bi) {
      constexpr int b = decltype(bi)::value;
      float2 s[A];
#pragma unroll
      for (int a = 0; a < A; ++a) s[a] = x[b + B * a];
      dft<A>(s);
      static_for<A>([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        z[b + B * a] = mul_root<b * a, R>(s[a]);
      });
    });
#pragma unroll
    for (int a = 0; a < A; ++a) {
      float2 s[B];
#pragma unroll
      for (int b = 0; b < B; ++b) s[b] = z[b + B * a];
      dft<B>(s);
#pragma unroll
      for (int b = 0; b < B; ++b) x[a + A * b] = s[b];
    }
  }
}

}  // namespace dft3d
