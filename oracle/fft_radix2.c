/*
 * O2 -- recursive radix-2 FFT in FP64.  TEST INFRASTRUCTURE ONLY (oracle.h).
 *
 * Section 2.1, eq. (3) with n = 2 * (n/2): the length-n DFT splits into two
 * half-length DFTs of the even- and odd-indexed samples (stage I), a
 * point-wise twiddle (stage II, eq. (4)) and length-2 DFTs across the
 * halves (stage IV); written as the textbook decimation-in-time recursion
 *   E = FFT(x[0::2]), O = FFT(x[1::2]),
 *   y[k] = E[k] + w^k O[k],  y[k + n/2] = E[k] - w^k O[k],  k < n/2,
 * with w = exp(sign * 2*pi*i / n).  Each w^k is taken directly from cos/sin
 * of the C library (no recurrence), once per length, and shared by every
 * level through w_m^k = w_n^{k n / m}.  The 3D transform applies this along
 * axis 2, then 1, then 0 (Section 2.3).  This file shares no code with
 * dft_direct.c.  parity pinned: equal to O1 and to closed forms in
 * tests/test_oracle.py.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double kTau = 6.283185307179586476925286766559;

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* R[k] = exp(sign * 2 pi i k / n) for k < n/2 (or one entry when n == 1). */
static double* half_roots(int64_t n, int sign) {
  int64_t h = n / 2 > 0 ? n / 2 : 1;
  double* r = (double*)malloc(sizeof(double) * 2 * (size_t)h);
  if (!r) return NULL;
  for (int64_t k = 0; k < h; ++k) {
    double a = kTau * (double)k / (double)n;
    r[2 * k] = cos(a);
    r[2 * k + 1] = (double)sign * sin(a);
  }
  return r;
}

/* out[0..m) = DFT_m of in[0], in[s], ..., in[(m-1) s]; R holds the roots of
 * the top-level length n, so w_m^k = R[k * (n / m)]. */
static void fft_rec(const double* in, int64_t s, double* out, int64_t m,
                    const double* R, int64_t n) {
  if (m == 1) {
    out[0] = in[0];
    out[1] = in[1];
    return;
  }
  int64_t h = m / 2;
  fft_rec(in, 2 * s, out, h, R, n);             /* even samples -> out[0..h) */
  fft_rec(in + 2 * s, 2 * s, out + 2 * h, h, R, n); /* odd -> out[h..m) */
  int64_t step = n / m;
  for (int64_t k = 0; k < h; ++k) {
    double wr = R[2 * k * step], wi = R[2 * k * step + 1];
    double er = out[2 * k], ei = out[2 * k + 1];
    double orr = out[2 * (k + h)], oi = out[2 * (k + h) + 1];
    double tr = wr * orr - wi * oi, ti = wr * oi + wi * orr;
    out[2 * k] = er + tr;
    out[2 * k + 1] = ei + ti;
    out[2 * (k + h)] = er - tr;
    out[2 * (k + h) + 1] = ei - ti;
  }
}

int oracle_fft1d_radix2(const double* x, double* y, int64_t n, int sign) {
  if (!is_pow2(n) || (sign != 1 && sign != -1) || !x || !y || x == y) return -1;
  double* R = half_roots(n, sign);
  if (!R) return -2;
  fft_rec(x, 1, y, n, R, n);
  free(R);
  return 0;
}

/* Geometry of the pencils along one axis of a C-order (n0, n1, n2) array:
 * pencil p (0 <= p < count) starts at (p / inner) * outer_stride + p % inner
 * and has element stride `stride`. */
typedef struct {
  int64_t n, stride, count, inner, outer_stride;
} axis_geom;

static axis_geom geom(int64_t n0, int64_t n1, int64_t n2, int axis) {
  axis_geom g;
  if (axis == 2) {
    g.n = n2; g.stride = 1; g.count = n0 * n1; g.inner = 1; g.outer_stride = n2;
  } else if (axis == 1) {
    g.n = n1; g.stride = n2; g.count = n0 * n2; g.inner = n2; g.outer_stride = n1 * n2;
  } else {
    g.n = n0; g.stride = n1 * n2; g.count = n1 * n2; g.inner = n1 * n2; g.outer_stride = 0;
  }
  return g;
}

static int fft_axis(double* y, int64_t n0, int64_t n1, int64_t n2, int axis,
                    int sign) {
  axis_geom g = geom(n0, n1, n2, axis);
  double* R = half_roots(g.n, sign);
  if (!R) return -2;
  int failed = 0;
#pragma omp parallel
  {
    double* buf = (double*)malloc(sizeof(double) * 4 * (size_t)g.n);
    if (!buf) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(static)
    for (int64_t p = 0; p < g.count; ++p) {
      if (!buf) continue;
      int64_t base = (p / g.inner) * g.outer_stride + p % g.inner;
      double* v = buf;
      double* o = buf + 2 * g.n;
      for (int64_t j = 0; j < g.n; ++j) {
        v[2 * j] = y[2 * (base + j * g.stride)];
        v[2 * j + 1] = y[2 * (base + j * g.stride) + 1];
      }
      fft_rec(v, 1, o, g.n, R, g.n);
      for (int64_t k = 0; k < g.n; ++k) {
        y[2 * (base + k * g.stride)] = o[2 * k];
        y[2 * (base + k * g.stride) + 1] = o[2 * k + 1];
      }
    }
    free(buf);
  }
  free(R);
  return failed ? -2 : 0;
}

int oracle_fft3d_radix2(const double* x, double* y, int64_t n0, int64_t n1,
                        int64_t n2, int sign) {
  if (!is_pow2(n0) || !is_pow2(n1) || !is_pow2(n2) ||
      (sign != 1 && sign != -1) || !x || !y)
    return -1;
  if (y != x) memcpy(y, x, sizeof(double) * 2 * (size_t)(n0 * n1 * n2));
  for (int axis = 2; axis >= 0; --axis) {
    int rc = fft_axis(y, n0, n1, n2, axis, sign);
    if (rc) return rc;
  }
  return 0;
}

int oracle_fft_pencils_radix2(const float* x, int64_t n0, int64_t n1,
                              int64_t n2, int axis, int sign, int64_t first,
                              int64_t count, double* out) {
  if (!is_pow2(n0) || !is_pow2(n1) || !is_pow2(n2) || axis < 0 || axis > 2 ||
      (sign != 1 && sign != -1) || !x || !out || first < 0 || count < 0)
    return -1;
  axis_geom g = geom(n0, n1, n2, axis);
  if (first + count > g.count) return -1;
  double* R = half_roots(g.n, sign);
  if (!R) return -2;
  int failed = 0;
#pragma omp parallel
  {
    double* v = (double*)malloc(sizeof(double) * 2 * (size_t)g.n);
    if (!v) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(static)
    for (int64_t c = 0; c < count; ++c) {
      if (!v) continue;
      int64_t p = first + c;
      int64_t base = (p / g.inner) * g.outer_stride + p % g.inner;
      for (int64_t j = 0; j < g.n; ++j) {
        v[2 * j] = (double)x[2 * (base + j * g.stride)];
        v[2 * j + 1] = (double)x[2 * (base + j * g.stride) + 1];
      }
      fft_rec(v, 1, out + 2 * c * g.n, g.n, R, g.n);
    }
    free(v);
  }
  free(R);
  return failed ? -2 : 0;
}
