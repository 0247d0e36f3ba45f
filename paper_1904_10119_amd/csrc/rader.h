// Prime lengths n whose n - 1 has no prime factor above 13: the DFT of
// length n as a cyclic convolution of length L = n - 1 (Rader's
// identity), computed with two mixed-radix FFTs of length L.
//
// With g a generator of the multiplicative group mod n, every nonzero index
// is a power of g: for k = g^-p and j = g^q,
//   y[g^-p] = x[0] + sum_q x[g^q] w_n^(g^(q - p)),
// a cyclic convolution (over q) of a[q] = x[g^q] with b[m] = w_n^(g^-m).
// Through FFTs of length L: C = FFT_L(a) * FFT_L(b) / L, and the inverse FFT
// read backwards, c[p] = FFT_L(C)[(L - p) mod L].  Since g^-p = g^(L - p),
// the output sits at y[g^j] = x[0] + FFT_L(C)[j]: the same permutation as
// the input.  The zero frequency is y[0] = x[0] + FFT_L(a)[0].
//
// One workgroup takes a tile of T pencils through the chain in LDS, like
// the mixed-radix pass (mixed_kernel.h, whose stage code it reuses): load
// the n inputs (lanes along the pencil), gather a[j] = x[g^j] into the
// first stage of FFT_L, the later stages, keep FFT_L(a)[0], multiply by
// FFT_L(b) / L, the second FFT_L, scatter x[0] + FFT_L(C)[j] to g^j, and
// store the n outputs rotated (T consecutive pencils per output row).
//
// PassArgs fields used: pencil fields and element strides as for every
// pass, res_mask = n, twp_mask = the radix code of L (mixed_kernel.h).
// Tables: tw = the stage twiddles of L (mixed-radix layout); twp =
// FFT_L(b) / L (L entries, FP64-built) followed by the generator powers
// g^j mod n (j < L) as 32-bit integers.
#pragma once

#include "mixed_kernel.h"

namespace dft3d {

// LDS of a tile: the pencils, the per-pencil x[0] and FFT_L(a)[0], then
// where two workgroups per CU still fit the generator powers (else read
// from global memory) and the stage twiddles.
template <int T, int NMAX> constexpr int rader_lds_bytes(bool perm, bool twl) {
  return (T * NMAX + 2 * T + (twl ? NMAX : 0)) * 8 + (perm ? NMAX * 4 : 0);
}
template <int T, int NMAX> constexpr bool rader_perm_in_lds() {
  return 2 * rader_lds_bytes<T, NMAX>(true, false) <= 160 * 1024;
}
template <int T, int NMAX> constexpr bool rader_twiddles_in_lds() {
  return 2 * rader_lds_bytes<T, NMAX>(rader_perm_in_lds<T, NMAX>(), true) <= 160 * 1024;
}

template <int T, int NMAX, int TH, int VAR>
__global__ void __launch_bounds__(TH)
rader_axis_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                  const float2* __restrict__ twp, const PassArgs a) {
  constexpr int P = TH / T;   // threads per pencil
  constexpr int V = NMAX / P; // points per thread
  constexpr bool COMP = VAR == 1 && NMAX <= 2048;
  constexpr bool PL = rader_perm_in_lds<T, NMAX>();
  constexpr bool TWL = rader_twiddles_in_lds<T, NMAX>();
  __shared__ float2 buf[T * NMAX + (TWL ? NMAX : 0)];
  __shared__ int lperm_store[PL ? NMAX : 1];
  __shared__ float2 x0s[T], dcs[T];
  const int n = (int)a.res_mask;  // prime, n + 1 <= NMAX
  const int L = n - 1;
  const int sq = n + 1;
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  const int q = tid / P, p = tid % P;
  float2* pen = buf + q * sq;
  const float2* twv = TWL ? buf + T * NMAX : tw;
  const float2* __restrict__ bl = twp;
  const int* __restrict__ perm = reinterpret_cast<const int*>(twp + L);
  if constexpr (TWL) {  // the stage twiddles of L (L - 1 entries)
    float2* tl = buf + T * NMAX;
#pragma unroll
    for (int i = 0; i < (NMAX + TH - 1) / TH; ++i) {
      const int j = tid + TH * i;
      if (j < L - 1) tl[j] = tw[j];
    }
  }
  const int* lperm = PL ? lperm_store : perm;
  if constexpr (PL) {
#pragma unroll
    for (int i = 0; i < (NMAX + TH - 1) / TH; ++i) {
      const int j = tid + TH * i;
      if (j < L) lperm_store[j] = perm[j];
    }
  }
  {  // the pencil into LDS, lanes along it (pencils past the end of a ragged
     // last tile read the last pencil)
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    const float2* s = src + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int k = p + P * i;
      if (k < n) {
        float2 x = s[(int64_t)k * a.ijs];
        if (a.conj_in) x.y = -x.y;
        pen[k] = x;
      }
    }
  }
  __syncthreads();  // inputs, twiddles and powers in LDS
  if (p == 0) x0s[q] = pen[0];
  uint64_t code0 = (uint64_t)a.twp_mask;
  const int R0 = (int)(code0 & 255);
  code0 >>= 8;
  // FFT_L of a[j] = x[g^j]: the first stage gathers through the powers
  with_radix<VAR, COMP>(R0, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    constexpr int K = (V + R - 1) / R;
    const int nr = L / R;
    float2 v[K][R];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int t = p + P * i;
      if (t < nr) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = pen[lperm[t + r * nr]];
      }
    }
    __syncthreads();  // every input is read before the stage writes
    mixed_first_compute<R, V>(v, 0, pen, L, p, P);
  });
  int ns = R0;
  for (uint64_t c = code0; c; c >>= 8) {
    const int R = (int)(c & 255);
    with_radix<VAR, COMP>(R, [&](auto rc) {
      mixed_stage<decltype(rc)::value, V>(pen, L, ns, twv, p, P);
    });
    ns *= R;
  }
  // keep FFT_L(a)[0] (the same thread owns k = 0 below), times FFT_L(b) / L
  if (p == 0) dcs[q] = pen[0];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int k = p + P * i;
    if (k < L) pen[k] = cmul(pen[k], bl[k]);
  }
  __syncthreads();
  // the second FFT_L, its first stage from LDS
  with_radix<VAR, COMP>(R0, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    float2 v[(V + R - 1) / R][R];
    mixed_first_load<R, V>(v, pen, 1, L, p, P);
    __syncthreads();
    mixed_first_compute<R, V>(v, 0, pen, L, p, P);
  });
  ns = R0;
  for (uint64_t c = code0; c; c >>= 8) {
    const int R = (int)(c & 255);
    with_radix<VAR, COMP>(R, [&](auto rc) {
      mixed_stage<decltype(rc)::value, V>(pen, L, ns, twv, p, P);
    });
    ns *= R;
  }
  // y[g^j] = x[0] + FFT_L(C)[j], y[0] = x[0] + FFT_L(a)[0], in LDS
  {
    const float2 x0 = x0s[q];
    float2 d[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int j = p + P * i;
      if (j < L) d[i] = cadd(x0, pen[j]);
    }
    __syncthreads();  // every FFT output is read before the scatter
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int j = p + P * i;
      if (j < L) pen[lperm[j]] = d[i];
    }
    if (p == 0) pen[0] = cadd(x0, dcs[q]);
  }
  __syncthreads();
  // rotated store: thread on pencil tid mod T, outputs k = tid / T + KS i
  const int qs = tid % T;
  const int64_t b = tile * T + qs;
  if (b < a.B) {
    float2* d = dst + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    const float2* ps = buf + qs * sq;
    constexpr int KS = TH / T;
#pragma unroll
    for (int i = 0; i < NMAX / KS; ++i) {
      const int k = tid / T + KS * i;
      if (k < n) {
        float2 w = ps[k];
        if (a.conj_out) w.y = -w.y;
        d[(int64_t)k * a.oks] = w;
      }
    }
  }
}

// The same pass for one prime N known at compile time, CODE the radix code
// of N - 1 (variant 1 radices): stage sizes and offsets fold into constants
// and the radix switch disappears, which keeps the kernel's registers low
// enough for two workgroups per CU.
template <int T, int NMAX, int TH, int N, uint64_t CODE>
__global__ void __launch_bounds__(TH)
rader_axis_fixed(const float2* src, float2* dst, const float2* __restrict__ tw,
                 const float2* __restrict__ twp, const PassArgs a) {
  constexpr int P = TH / T;
  constexpr int V = NMAX / P;
  constexpr int L = N - 1;
  constexpr int SQ = N + 1;
  constexpr int R1 = (int)(CODE & 255);
  constexpr bool PL = rader_perm_in_lds<T, NMAX>();
  constexpr bool TWL = rader_twiddles_in_lds<T, NMAX>();
  static_assert(N + 1 <= NMAX, "length fits the tile");
  __shared__ float2 buf[T * NMAX + (TWL ? NMAX : 0)];
  __shared__ int lperm_store[PL ? NMAX : 1];
  __shared__ float2 x0s[T], dcs[T];
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  const int q = tid / P, p = tid % P;
  float2* pen = buf + q * SQ;
  const float2* twv = TWL ? buf + T * NMAX : tw;
  const float2* __restrict__ bl = twp;
  const int* __restrict__ perm = reinterpret_cast<const int*>(twp + L);
  if constexpr (TWL) {
    float2* tl = buf + T * NMAX;
#pragma unroll
    for (int i = 0; i < (NMAX + TH - 1) / TH; ++i) {
      const int j = tid + TH * i;
      if (j < L - 1) tl[j] = tw[j];
    }
  }
  const int* lperm = PL ? lperm_store : perm;
  if constexpr (PL) {
#pragma unroll
    for (int i = 0; i < (NMAX + TH - 1) / TH; ++i) {
      const int j = tid + TH * i;
      if (j < L) lperm_store[j] = perm[j];
    }
  }
  {
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    const float2* s = src + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int k = p + P * i;
      if (k < N) {
        float2 x = s[(int64_t)k * a.ijs];
        if (a.conj_in) x.y = -x.y;
        pen[k] = x;
      }
    }
  }
  __syncthreads();
  if (p == 0) x0s[q] = pen[0];
  {  // FFT_L of a[j] = x[g^j]
    constexpr int K = (V + R1 - 1) / R1;
    constexpr int NR = L / R1;
    float2 v[K][R1];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int t = p + P * i;
      if (t < NR) {
#pragma unroll
        for (int r = 0; r < R1; ++r) v[i][r] = pen[lperm[t + r * NR]];
      }
    }
    __syncthreads();
    mixed_first_compute<R1, V>(v, 0, pen, L, p, P);
  }
  mixed_stages_fixed<(CODE >> 8), R1, V, L>(pen, twv, p, P);
  if (p == 0) dcs[q] = pen[0];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int k = p + P * i;
    if (k < L) pen[k] = cmul(pen[k], bl[k]);
  }
  __syncthreads();
  {
    float2 v[(V + R1 - 1) / R1][R1];
    mixed_first_load<R1, V>(v, pen, 1, L, p, P);
    __syncthreads();
    mixed_first_compute<R1, V>(v, 0, pen, L, p, P);
  }
  mixed_stages_fixed<(CODE >> 8), R1, V, L>(pen, twv, p, P);
  {
    const float2 x0 = x0s[q];
    float2 d[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int j = p + P * i;
      if (j < L) d[i] = cadd(x0, pen[j]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int j = p + P * i;
      if (j < L) pen[lperm[j]] = d[i];
    }
    if (p == 0) pen[0] = cadd(x0, dcs[q]);
  }
  __syncthreads();
  const int qs = tid % T;
  const int64_t b = tile * T + qs;
  if (b < a.B) {
    float2* d = dst + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    const float2* ps = buf + qs * SQ;
    constexpr int KS = TH / T;
#pragma unroll
    for (int i = 0; i < NMAX / KS; ++i) {
      const int k = tid / T + KS * i;
      if (k < N) {
        float2 w = ps[k];
        if (a.conj_out) w.y = -w.y;
        d[(int64_t)k * a.oks] = w;
      }
    }
  }
}

template <int T, int NMAX, int TH, int N, uint64_t CODE>
hipError_t launch_rader_fixed(const PassArgs& a, const float2* src, float2* dst,
                              const float2* tw, const float2* twp, hipStream_t stream) {
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (a.res_mask != N || (uint64_t)a.twp_mask != CODE) return hipErrorInvalidValue;
  hipLaunchKernelGGL((rader_axis_fixed<T, NMAX, TH, N, CODE>), dim3((unsigned)blocks), dim3(TH),
                     0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int T, int NMAX, int TH, int N, uint64_t CODE>
KernelInfo kernel_info_rader_fixed() {
  constexpr int LDS =
      rader_lds_bytes<T, NMAX>(rader_perm_in_lds<T, NMAX>(), rader_twiddles_in_lds<T, NMAX>());
  static_assert(2 * LDS <= 160 * 1024, "two workgroups per CU");
  KernelInfo k{NMAX, T, MODE_ROW, MODE_COL, 0, TH, LDS,
               &launch_rader_fixed<T, NMAX, TH, N, CODE>, 0, 0};
  k.rader = 1;
  k.fixed_n = N;
  k.fixed_code = CODE;
  return k;
}

template <int T, int NMAX, int TH, int VAR>
hipError_t launch_rader(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                        const float2* twp, hipStream_t stream) {
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (a.res_mask < 3 || a.res_mask + 1 > NMAX ||
      !mixed_kernel_runs(VAR, NMAX, (uint64_t)a.twp_mask))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((rader_axis_kernel<T, NMAX, TH, VAR>), dim3((unsigned)blocks), dim3(TH), 0,
                     stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int T, int NMAX, int TH, int VAR>
KernelInfo kernel_info_rader() {
  constexpr int LDS =
      rader_lds_bytes<T, NMAX>(rader_perm_in_lds<T, NMAX>(), rader_twiddles_in_lds<T, NMAX>());
  static_assert(2 * LDS <= 160 * 1024, "two workgroups per CU");
  static_assert(TH % T == 0 && NMAX % (TH / T) == 0 && TH <= 1024, "tile shape");
  KernelInfo k{NMAX, T, MODE_ROW, MODE_COL, 0, TH, LDS, &launch_rader<T, NMAX, TH, VAR>, 0, 0};
  k.rader = VAR;
  return k;
}

}  // namespace dft3d
