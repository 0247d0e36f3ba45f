/*
 * O1 -- direct FP64 DFT.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Section 2.1, eq. (1): y = DFT_n x, a dense matrix-vector product.
 * Section 2.1, eq. (2): DFT_n[l][k] = w_n^{l k}.  The printed root of unity
 * is garbled; it is read as w_n = exp(-2*pi*i/n) for the forward transform,
 * and exp(+2*pi*i/n) for the inverse (sign = +1), which is left unscaled.
 * Section 2.3: the n-D DFT is 1D DFTs applied along every dimension, so the
 * 3D transform applies the 1D product along axis 2, axis 1 and axis 0.
 *
 * Every output entry is the plain sum over j in ascending order of
 * v[j] * W[(j*k) mod n] with W[m] = cos(2 pi m/n) + sign*i*sin(2 pi m/n)
 * from the C library; (j*k) mod n is reduced in 64-bit integers so that the
 * phase is exact.  parity pinned: closed forms, brute force and invariants
 * in tests/test_oracle.py.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double kTwoPi = 6.283185307179586476925286766559;

/* W[m] = w_n^m for m < n, interleaved. */
static double* make_roots(int64_t n, int sign) {
  double* w = (double*)malloc(sizeof(double) * 2 * (size_t)n);
  if (!w) return NULL;
  for (int64_t m = 0; m < n; ++m) {
    double a = kTwoPi * (double)m / (double)n;
    w[2 * m] = cos(a);
    w[2 * m + 1] = (double)sign * sin(a);
  }
  return w;
}

/* out[k] = sum_j v[j] * W[(j*k) mod n]; v, out: 2n doubles, distinct. */
static void dft_vec(const double* v, double* out, int64_t n, const double* W) {
  for (int64_t k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      int64_t m = (j * k) % n;
      double wr = W[2 * m], wi = W[2 * m + 1];
      double vr = v[2 * j], vi = v[2 * j + 1];
      sr += vr * wr - vi * wi;
      si += vr * wi + vi * wr;
    }
    out[2 * k] = sr;
    out[2 * k + 1] = si;
  }
}

int oracle_dft1d_direct(const double* x, double* y, int64_t n, int sign) {
  if (n <= 0 || (sign != 1 && sign != -1) || !x || !y) return -1;
  double* W = make_roots(n, sign);
  if (!W) return -2;
  dft_vec(x, y, n, W);
  free(W);
  return 0;
}

/* Apply the direct 1D DFT along one axis of a (n0,n1,n2) array in place.
 * The pencil along `axis` through (a, b) -- a, b the two other indices --
 * starts at base and has element stride `stride`. */
static int direct_axis(double* y, int64_t n0, int64_t n1, int64_t n2, int axis,
                       int sign) {
  int64_t n, stride, outer, inner, outer_stride;
  if (axis == 2) { n = n2; stride = 1;       outer = n0 * n1; inner = 1;  outer_stride = n2; }
  else if (axis == 1) { n = n1; stride = n2; outer = n0; inner = n2; outer_stride = n1 * n2; }
  else { n = n0; stride = n1 * n2; outer = 1; inner = n1 * n2; outer_stride = 0; }
  double* W = make_roots(n, sign);
  if (!W) return -2;
  int failed = 0;
#pragma omp parallel
  {
    double* v = (double*)malloc(sizeof(double) * 4 * (size_t)n);
    if (!v) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(static)
    for (int64_t p = 0; p < outer * inner; ++p) {
      if (!v) continue;
      int64_t a = p / inner, b = p % inner;
      int64_t base = a * outer_stride + b;
      double* out = v + 2 * n;
      for (int64_t j = 0; j < n; ++j) {
        v[2 * j] = y[2 * (base + j * stride)];
        v[2 * j + 1] = y[2 * (base + j * stride) + 1];
      }
      dft_vec(v, out, n, W);
      for (int64_t k = 0; k < n; ++k) {
        y[2 * (base + k * stride)] = out[2 * k];
        y[2 * (base + k * stride) + 1] = out[2 * k + 1];
      }
    }
    free(v);
  }
  free(W);
  return failed ? -2 : 0;
}

int oracle_dft3d_direct(const double* x, double* y, int64_t n0, int64_t n1,
                        int64_t n2, int sign) {
  if (n0 <= 0 || n1 <= 0 || n2 <= 0 || (sign != 1 && sign != -1) || !x || !y)
    return -1;
  size_t total = (size_t)(n0 * n1 * n2);
  if (y != x) memcpy(y, x, sizeof(double) * 2 * total);
  for (int axis = 2; axis >= 0; --axis) {
    int rc = direct_axis(y, n0, n1, n2, axis, sign);
    if (rc) return rc;
  }
  return 0;
}

int oracle_dft3d_sample_pencils(const float* x, int64_t n0, int64_t n1,
                                int64_t n2, int sign, const int64_t* k0,
                                const int64_t* k1, int64_t nsamp,
                                double* out) {
  if (n0 <= 0 || n1 <= 0 || n2 <= 0 || (sign != 1 && sign != -1) || !x ||
      !k0 || !k1 || !out || nsamp < 0)
    return -1;
  for (int64_t s = 0; s < nsamp; ++s)
    if (k0[s] < 0 || k0[s] >= n0 || k1[s] < 0 || k1[s] >= n1) return -1;
  double* W0 = make_roots(n0, sign);
  double* W1 = make_roots(n1, sign);
  double* W2 = make_roots(n2, sign);
  double* z = (double*)calloc((size_t)(2 * n2 * (nsamp > 0 ? nsamp : 1)),
                              sizeof(double));
  int rc = 0;
  if (!W0 || !W1 || !W2 || !z) {
    rc = -2;
  } else {
    /* z_s[i2] = sum over (i0, i1) in ascending order of
     * x[i0,i1,i2] * w0^{i0 k0} * w1^{i1 k1}.  One sweep over x serves every
     * sample; each thread owns a contiguous range of i2, so every z entry is
     * summed by one thread in a fixed order. */
#pragma omp parallel
    {
      int64_t nt = 1, t = 0;
#ifdef _OPENMP
      nt = omp_get_num_threads();
      t = omp_get_thread_num();
#endif
      int64_t lo = n2 * t / nt, hi = n2 * (t + 1) / nt;
      for (int64_t i0 = 0; i0 < n0 && lo < hi; ++i0) {
        for (int64_t i1 = 0; i1 < n1; ++i1) {
          const float* row = x + 2 * (size_t)((i0 * n1 + i1) * n2);
          for (int64_t s = 0; s < nsamp; ++s) {
            int64_t m0 = (i0 * k0[s]) % n0, m1 = (i1 * k1[s]) % n1;
            double ar = W0[2 * m0], ai = W0[2 * m0 + 1];
            double br = W1[2 * m1], bi = W1[2 * m1 + 1];
            double cr = ar * br - ai * bi, ci = ar * bi + ai * br;
            double* zs = z + 2 * s * n2;
            for (int64_t i2 = lo; i2 < hi; ++i2) {
              double xr = (double)row[2 * i2], xi = (double)row[2 * i2 + 1];
              zs[2 * i2] += xr * cr - xi * ci;
              zs[2 * i2 + 1] += xr * ci + xi * cr;
            }
          }
        }
      }
    }
    for (int64_t s = 0; s < nsamp; ++s)
      dft_vec(z + 2 * s * n2, out + 2 * s * n2, n2, W2);
  }
  free(W0);
  free(W1);
  free(W2);
  free(z);
  return rc;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
