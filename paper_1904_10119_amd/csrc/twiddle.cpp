// Twiddle tables: the only FP64 step of the library.
//
// w_n^m = exp(-2 pi i m / n) (eq. (4) entries, forward direction).  The
// exponent is reduced exactly in integers to a whole number of quarter turns
// plus an angle in [0, pi/2); that angle is folded into [0, pi/4] so the C
// library's cos and sin are called only on small arguments, and 0, +-1 and
// +-sqrt(1/2) are exact.  Each entry is rounded once to FP32.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/dft3d.h"
#include "internal.h"

namespace dft3d {

void root_fp64(int64_t m, int64_t n, double& c, double& s) {
  const double half_pi = 1.57079632679489661923132169163975144;
  m %= n;
  if (m < 0) m += n;
  const int64_t q = (4 * m) / n;      // quarter turns
  const int64_t rem = 4 * m - q * n;  // (pi/2) * rem / n left over
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
}

void make_roots(int64_t n, float2* out) {
  for (int64_t m = 0; m < n; ++m) {
    double c, s;
    root_fp64(m, n, c, s);
    out[m] = make_float2((float)c, (float)(-s));
  }
}

namespace {

// Round to the nearest value with `bits` significand bits (ties to even),
// with the smallest quantum `minq` (subnormal spacing); exact in FP64.
double round_sig(double v, int bits, double minq) {
  if (v == 0.0) return 0.0;
  int e;
  std::frexp(v, &e);                      // |v| in [2^(e-1), 2^e)
  double q = std::ldexp(1.0, e - bits);   // spacing of the format at v
  if (q < minq) q = minq;
  return std::nearbyint(v / q) * q;       // default rounding: ties to even
}

unsigned short bf16_bits(double v) {  // v exactly representable in bf16
  const float f = (float)v;
  unsigned int u;
  std::memcpy(&u, &f, 4);
  return (unsigned short)(u >> 16);
}

unsigned short f16_bits(double v) {  // v exactly representable in fp16
  const _Float16 h = (_Float16)v;
  unsigned short u;
  std::memcpy(&u, &h, 2);
  return u;
}

}  // namespace

// Lane l of the 16x16x32 MFMA holds A[l % 16][8 (l / 16) + i].  Length-16
// leaf: matrix 0 is [Fr | -Fi], matrix 1 is [Fi | Fr] with F[m][k] =
// w_16^{m k} (forward).
// Each entry is split from FP64: bf16 terms unscaled, fp16 terms scaled by
// 2^(11 t) so that the small terms stay normal.
void make_leaf_table(int precision, unsigned short* out) {
  const bool fp16 = precision == DFT3D_PREC_FP16X1 || precision == DFT3D_PREC_FP16X3;
  for (int t = 0; t < 3; ++t)
    for (int c = 0; c < 2; ++c)
      for (int lane = 0; lane < 64; ++lane)
        for (int i = 0; i < 8; ++i) {
          const int m = lane % 16, k = 8 * (lane / 16) + i, col = k % 16;
          double cs, sn;
          root_fp64((int64_t)m * col, 16, cs, sn);
          const double fr = cs, fi = -sn;  // w_16^{m col} = cos - i sin
          double v;
          if (c == 0) v = k < 16 ? fr : -fi;
          else v = k < 16 ? fi : fr;
          // peel terms 0 .. t
          double r = v, h = 0.0;
          for (int j = 0; j <= t; ++j) {
            h = fp16 ? round_sig(r, 11, std::ldexp(1.0, -24)) : round_sig(r, 8, 0.0);
            r = fp16 ? (r - h) * 2048.0 : r - h;
          }
          out[((t * 2 + c) * 64 + lane) * 8 + i] = fp16 ? f16_bits(h) : bf16_bits(h);
        }
  // Length-32 leaf, odd-half table: H[p][k] = w_32^{p (2k + 1)} (p, k < 16),
  // matrix 0 [Hr | -Hi], matrix 1 [Hi | Hr].
  unsigned short* out32 = out + 3 * 2 * 64 * 8;
  for (int t = 0; t < 3; ++t)
    for (int c = 0; c < 2; ++c)
      for (int lane = 0; lane < 64; ++lane)
        for (int i = 0; i < 8; ++i) {
          const int p = lane % 16, k = 8 * (lane / 16) + i, col = k % 16;
          double cs, sn;
          root_fp64((int64_t)p * (2 * col + 1), 32, cs, sn);
          const double hr = cs, hi = -sn;  // w_32^{p (2 col + 1)} = cos - i sin
          double v;
          if (c == 0) v = k < 16 ? hr : -hi;
          else v = k < 16 ? hi : hr;
          double r = v, h = 0.0;
          for (int j = 0; j <= t; ++j) {
            h = fp16 ? round_sig(r, 11, std::ldexp(1.0, -24)) : round_sig(r, 8, 0.0);
            r = fp16 ? (r - h) * 2048.0 : r - h;
          }
          out32[((t * 2 + c) * 64 + lane) * 8 + i] = fp16 ? f16_bits(h) : bf16_bits(h);
        }
}

namespace {
int64_t mul_mod(int64_t a, int64_t b, int64_t n) { return (a * b) % n; }

// The smallest generator of the multiplicative group mod the prime n.
int64_t rader_generator(int64_t n) {
  std::vector<int64_t> f;  // prime factors of n - 1
  int64_t m = n - 1;
  for (int64_t d = 2; d * d <= m; ++d)
    if (m % d == 0) {
      f.push_back(d);
      while (m % d == 0) m /= d;
    }
  if (m > 1) f.push_back(m);
  for (int64_t g = 2; g < n; ++g) {
    bool gen = true;
    for (int64_t p : f) {
      int64_t e = (n - 1) / p, r = 1, base = g;
      while (e) {  // g^((n - 1) / p) mod n
        if (e & 1) r = mul_mod(r, base, n);
        base = mul_mod(base, base, n);
        e >>= 1;
      }
      if (r == 1) {
        gen = false;
        break;
      }
    }
    if (gen) return g;
  }
  return 0;
}
}  // namespace

int64_t rader_table_size(int64_t n) { return (n - 1) + (n - 1 + 1) / 2; }

void make_rader_tables(int64_t n, float2* out) {
  const int64_t L = n - 1, g = rader_generator(n);
  std::vector<int64_t> pw(L);
  pw[0] = 1;
  for (int64_t j = 1; j < L; ++j) pw[j] = mul_mod(pw[j - 1], g, n);
  // b[m] = w_n^(g^-m) = w_n^(g^((L - m) mod L)), B = DFT_L(b) in FP64
  std::vector<double> br(L), bi(L), cr(L), ci(L);
  for (int64_t m = 0; m < L; ++m) {
    double c, s;
    root_fp64(pw[(L - m) % L], n, c, s);
    br[m] = c;
    bi[m] = -s;
  }
  for (int64_t k = 0; k < L; ++k) root_fp64(k, L, cr[k], ci[k]);  // w_L^k = cr - i ci
  for (int64_t k = 0; k < L; ++k) {
    double sr = 0.0, si = 0.0;
    for (int64_t m = 0; m < L; ++m) {
      const int64_t e = (m * k) % L;
      const double wr = cr[e], wi = -ci[e];
      sr += br[m] * wr - bi[m] * wi;
      si += br[m] * wi + bi[m] * wr;
    }
    out[k] = make_float2((float)(sr / (double)L), (float)(si / (double)L));
  }
  int32_t* perm = reinterpret_cast<int32_t*>(out + L);
  for (int64_t j = 0; j < L; ++j) perm[j] = (int32_t)pw[j];
  if (L % 2) perm[L] = 0;  // the last slot's second half
}

int64_t bluestein_length(int64_t n) {
  int64_t m = 1;
  while (m < 2 * n - 1) m <<= 1;
  return m;
}

// w[j] = exp(-pi i j^2 / n) = w_{2n}^{j^2 mod 2n}, the exponent reduced in
// integers before the FP64 root.
void make_chirp(int64_t n, float2* out) {
  for (int64_t j = 0; j < n; ++j) {
    double c, s;
    root_fp64((j * j) % (2 * n), 2 * n, c, s);
    out[j] = make_float2((float)c, (float)(-s));
  }
}

void make_bluestein_filter(int64_t n, float2* out) {
  const int64_t m = bluestein_length(n);
  // wrapped filter h[d] = conj(w[|d|]) at d mod m, in FP64
  std::vector<double> hr(m, 0.0), hi(m, 0.0);
  for (int64_t d = 0; d < n; ++d) {
    double c, s;
    root_fp64((d * d) % (2 * n), 2 * n, c, s);  // w[d] = c - i s, conj = c + i s
    hr[d] = c;
    hi[d] = s;
    if (d > 0) {
      hr[m - d] = c;
      hi[m - d] = s;
    }
  }
  std::vector<double> rc(m), rs(m);
  for (int64_t l = 0; l < m; ++l) root_fp64(l, m, rc[l], rs[l]);
  for (int64_t l = 0; l < m; ++l) {
    double yr = 0.0, yi = 0.0;
    for (int64_t d = 0; d < m; ++d) {
      if (hr[d] == 0.0 && hi[d] == 0.0) continue;
      const int64_t e = (d * l) % m;  // exp(-2 pi i d l / m) = rc - i rs
      yr += hr[d] * rc[e] + hi[d] * rs[e];
      yi += hi[d] * rc[e] - hr[d] * rs[e];
    }
    out[l] = make_float2((float)(yr / (double)m), (float)(yi / (double)m));
  }
}

void make_mixed_twiddles(int64_t n, uint64_t code, float2* out) {
  int64_t ns = 1;
  for (uint64_t c = code; c; c >>= 8) {
    const int64_t R = (int64_t)(c & 255);
    for (int64_t r = 1; r < R; ++r)
      for (int64_t tm = 0; tm < ns; ++tm) {
        double cr, sr;
        root_fp64(tm * r, ns * R, cr, sr);
        out[(ns - 1) + (r - 1) * ns + tm] = make_float2((float)cr, (float)(-sr));
      }
    ns *= R;
  }
  if (ns != n) return;  // the code always multiplies to n (mixed_radix_code)
}

}  // namespace dft3d
