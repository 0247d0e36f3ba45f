/*
 * FP64 CPU oracle for the 3D complex DFT -- TEST INFRASTRUCTURE ONLY.
 *
 * This header is private to oracle/.  Nothing in the product library
 * (paper_1904_10119_amd/) includes it, links it or calls it; only tests/,
 * the smoke check and bench.py's CPU-baseline leg load liboracle.so.
 *
 * What is computed (Section 2.1, eqs. (1)-(2); Section 2.3, eqs. (6)-(8)):
 *   y[k0,k1,k2] = sum_{i0,i1,i2} x[i0,i1,i2] w0^{i0 k0} w1^{i1 k1} w2^{i2 k2},
 *   w_n = exp(sign * 2*pi*i / n), sign = -1 forward, +1 inverse (unnormalised).
 * Arrays are complex128, interleaved (re, im), C order (n0, n1, n2) with
 * n2 contiguous.
 *
 * Two independent methods live in separate source files with no shared code:
 *   O1  dft_direct.c  -- the 1D DFT as the matrix-vector product of eq. (1)
 *                        with the matrix of eq. (2), applied along each axis
 *                        (the n-D DFT as 1D DFTs along every dimension,
 *                        Section 2.3).
 *   O2  fft_radix2.c  -- recursive radix-2 decimation-in-time Cooley-Tukey
 *                        (the n = 2 * (n/2) case of eq. (3)), along each axis.
 *
 * Return value of every int function: 0 on success, -1 on bad arguments
 * (non-positive sizes, O2 with a non power-of-two length, sign not +-1),
 * -2 on allocation failure.  Outputs are written only on success.
 */
#ifndef DFT_ORACLE_H
#define DFT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- O1: direct summation (dft_direct.c) ---- */

/* y = DFT_n x for one vector of length n (eqs. (1)-(2)). x, y: 2n doubles;
 * x and y must not alias. */
int oracle_dft1d_direct(const double* x, double* y, int64_t n, int sign);

/* Full 3D DFT by direct 1D DFTs along axis 2, then 1, then 0.
 * x, y: 2*n0*n1*n2 doubles each; may alias (y == x is allowed). */
int oracle_dft3d_direct(const double* x, double* y, int64_t n0, int64_t n1,
                        int64_t n2, int sign);

/* Sampled output pencils for sizes where the full 3D result is too large:
 * for each pair (k0[s], k1[s]) computes y[k0,k1,0..n2-1] straight from the
 * definition: z[i2] = sum_{i0,i1} x[i0,i1,i2] w0^{i0 k0} w1^{i1 k1}, then a
 * direct DFT of z along i2.  x is complex64 (2*n0*n1*n2 floats, widened
 * exactly to FP64); out receives nsamp*n2 complex128 values. */
int oracle_dft3d_sample_pencils(const float* x, int64_t n0, int64_t n1,
                                int64_t n2, int sign, const int64_t* k0,
                                const int64_t* k1, int64_t nsamp,
                                double* out);

/* ---- O2: recursive radix-2 FFT (fft_radix2.c) ---- */

/* y = DFT_n x, n a power of two; x, y must not alias. */
int oracle_fft1d_radix2(const double* x, double* y, int64_t n, int sign);

/* Full 3D DFT by radix-2 FFTs along axis 2, then 1, then 0; y may alias x. */
int oracle_fft3d_radix2(const double* x, double* y, int64_t n0, int64_t n1,
                        int64_t n2, int sign);

/* O2 applied to `count` whole pencils along `axis` (0, 1 or 2) of a
 * complex64 array of shape (n0, n1, n2), starting at pencil index `first`
 * (pencils enumerated in C order over the two remaining axes).  Each pencil
 * is widened to FP64 and transformed; out receives count*len complex128
 * values (len = n_axis).  Used to time the oracle on a bounded sample of a
 * large workload and to check single pencils. */
int oracle_fft_pencils_radix2(const float* x, int64_t n0, int64_t n1,
                              int64_t n2, int axis, int sign, int64_t first,
                              int64_t count, double* out);

/* Number of OpenMP threads the oracle runs with. */
int oracle_num_threads(void);

/* Threads for later calls (timing on one core vs all host cores). */
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif

#endif
