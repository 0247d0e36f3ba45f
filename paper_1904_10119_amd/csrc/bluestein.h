// Lengths that are not powers of two: the DFT of length n as a circular
// convolution of length m (a power of two, m >= 2n - 1) computed with the
// power-of-two passes (Bluestein's chirp-z identity).  With the chirp
// w[j] = exp(-pi i j^2 / n) and jk = (j^2 + k^2 - (k - j)^2) / 2,
//   y[k] = w[k] sum_j (x[j] w[j]) conj(w[k - j]),
// so one axis step of the pencil rotation becomes five passes over a
// workspace of B pencils of length m:
//   pad     a[b][j] = x[b][j] w[j] (j < n), 0 (n <= j < m)
//   FFT_m   (a power-of-two pass kernel, rows in place)
//   filter  A[b][l] *= H[l] / m,  H = FFT_m of the wrapped filter conj(w[d]),
//           d in (-n, n)
//   FFT_m   (again; a forward DFT read backwards is the inverse DFT)
//   crop    y[k][b] = w[k] A'[b][(m - k) mod m] for k < n, written rotated
//           (k, b) like every pencil-schedule pass.
// The chirp and the filter come from FP64 tables built at plan time.
//
// PassArgs fields used: B = pencils; ijs = n; oks = m; conj_in / conj_out
// as for every pass (the inverse conjugates around the whole list).
#pragma once

#include "fft_device.h"
#include "internal.h"

namespace dft3d {

constexpr int kBluesteinThreads = 256;
constexpr int kBluesteinGridCap = 1 << 20;

__device__ __forceinline__ int ilog2_dev(int64_t v) { return 63 - __builtin_clzll(v); }

// pad: src pencils (B, n) contiguous -> dst (B, m); tw = chirp (n entries).
__global__ void __launch_bounds__(kBluesteinThreads)
bluestein_pad_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                     const float2* __restrict__ twp, const PassArgs a) {
  const int64_t n = a.ijs, m = a.oks;
  const int lm = ilog2_dev(m);
  const int64_t total = a.B << lm;
  for (int64_t idx = (int64_t)blockIdx.x * kBluesteinThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBluesteinThreads) {
    const int64_t b = idx >> lm, j = idx & (m - 1);
    float2 v = make_float2(0.f, 0.f);
    if (j < n) {
      v = src[b * n + j];
      if (a.conj_in) v.y = -v.y;
      v = cmul(v, tw[j]);
    }
    dst[idx] = v;
  }
}

// filter: (B, m) in place, times twp[l] = H[l] / m.
__global__ void __launch_bounds__(kBluesteinThreads)
bluestein_filter_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                        const float2* __restrict__ twp, const PassArgs a) {
  const int64_t m = a.oks;
  const int64_t total = a.B * m;
  for (int64_t idx = (int64_t)blockIdx.x * kBluesteinThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBluesteinThreads)
    dst[idx] = cmul(src[idx], twp[idx & (m - 1)]);
}

// crop: (B, m) -> dst (n, B): dst[k][b] = tw[k] src[b][(m - k) mod m], through
// a 32 x 32 LDS tile so that both the reads (along k) and the writes (along
// b) are contiguous.  One workgroup per tile, tiles k-fastest.
__global__ void __launch_bounds__(kBluesteinThreads)
bluestein_crop_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                      const float2* __restrict__ twp, const PassArgs a) {
  __shared__ float2 tile[32][33];
  const int64_t n = a.ijs, m = a.oks, B = a.B;
  const int64_t tiles_k = (n + 31) / 32;
  const int64_t t = blockIdx.x;
  const int64_t k0 = (t % tiles_k) * 32, b0 = (t / tiles_k) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
  for (int i = 0; i < 32; i += 8) {
    const int64_t b = b0 + ty + i, k = k0 + tx;
    if (b < B && k < n) tile[ty + i][tx] = src[b * m + ((m - k) & (m - 1))];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 32; i += 8) {
    const int64_t k = k0 + ty + i, b = b0 + tx;
    if (k < n && b < B) {
      float2 v = cmul(tile[tx][ty + i], tw[k]);
      if (a.conj_out) v.y = -v.y;
      dst[k * B + b] = v;
    }
  }
}

inline int64_t bluestein_grid(int64_t work) {
  int64_t g = (work + kBluesteinThreads - 1) / kBluesteinThreads;
  return g < 1 ? 1 : (g > kBluesteinGridCap ? kBluesteinGridCap : g);
}

inline hipError_t launch_bluestein_pad(const PassArgs& a, const float2* src, float2* dst,
                                       const float2* tw, const float2* twp, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  hipLaunchKernelGGL(bluestein_pad_kernel, dim3((unsigned)bluestein_grid(a.B * a.oks)),
                     dim3(kBluesteinThreads), 0, s, src, dst, tw, twp, a);
  return hipGetLastError();
}

inline hipError_t launch_bluestein_filter(const PassArgs& a, const float2* src, float2* dst,
                                          const float2* tw, const float2* twp, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  hipLaunchKernelGGL(bluestein_filter_kernel, dim3((unsigned)bluestein_grid(a.B * a.oks)),
                     dim3(kBluesteinThreads), 0, s, src, dst, tw, twp, a);
  return hipGetLastError();
}

inline hipError_t launch_bluestein_crop(const PassArgs& a, const float2* src, float2* dst,
                                        const float2* tw, const float2* twp, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  const int64_t tiles = ((a.ijs + 31) / 32) * ((a.B + 31) / 32);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(bluestein_crop_kernel, dim3((unsigned)tiles), dim3(kBluesteinThreads), 0,
                     s, src, dst, tw, twp, a);
  return hipGetLastError();
}

}  // namespace dft3d
