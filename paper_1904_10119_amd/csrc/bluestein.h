// Lengths that are not powers of two: the DFT of length n as a circular
// convolution of length m (a power of two, m >= 2n - 1) computed with two
// power-of-two FFTs (Bluestein's chirp-z identity).  With the chirp
// w[j] = exp(-pi i j^2 / n) and jk = (j^2 + k^2 - (k - j)^2) / 2,
//   y[k] = w[k] sum_j (x[j] w[j]) conj(w[k - j]),
// a circular convolution of the padded a[j] = x[j] w[j] (zero for j >= n)
// with the filter h[d] = conj(w[d]) wrapped to length m.  Writing the
// inverse DFT of length m as the forward one read backwards,
//   y[k] = w[k] FFT_m( FFT_m(a) * H / m )[(m - k) mod m],   H = FFT_m(h).
//
// One workgroup takes a tile of T pencils through the whole chain without
// leaving the chip: load the n inputs of each pencil (zeros above n) times
// the chirp, FFT_m, times H / m, FFT_m, and store output k < n times w[k]
// at its rotated place, like every pencil-schedule pass.  The first FFT
// ends in the row mapping (thread p of pencil q holds outputs p + P e),
// which is the input mapping of the second FFT, so the pencil stays in
// registers between the two; only the radix exchanges go through LDS.  The
// pass therefore moves n reads and n writes per pencil, as a power-of-two
// pass does.
//
// PassArgs fields used: pencil fields and element strides as for every
// pass (ijs along the input pencil, oks along the output), res_mask = n.
// Tables: tw = roots of length m; twp = the chirp (n entries) followed by
// H / m (m entries), both from FP64.
#pragma once

#include "pencil_index.h"

namespace dft3d {

// Convolution length 8192 (lengths 2049..4096): 32 elements per thread,
// radices 32, 16, 16; two pencils per workgroup fill 135 KB of LDS.
template <> struct Blocking<8192> {
  static constexpr int E = 32, R0 = 32, R1 = 16, R2 = 16;
};

// Stage twiddles laid out per stage for LDS: for each twiddled radix stage
// (ns, R) of the blocking, in order, entry (r - 1) ns + tm holds
// w_M^{tm r M / (ns R)} (r = 1 .. R-1, tm < ns), so the lanes of a wave, whose
// tm are consecutive, read consecutive entries.  M - R0 entries in all.
template <int M, class BL> constexpr int stage_table_size() {
  constexpr int NST = num_stages<BL>();
  return NST == 1 ? 0 : (NST == 2 ? (BL::R1 - 1) * BL::R0
                                  : (BL::R1 - 1) * BL::R0 + (BL::R2 - 1) * BL::R0 * BL::R1);
}

// Index into the roots of length M of stage-table entry j.
template <int M, class BL>
__device__ __forceinline__ int stage_table_root(int j) {
  constexpr int R0 = BL::R0, R1 = BL::R1, R2 = BL::R2, S1 = (R1 - 1) * R0;
  if (j < S1) return (j % R0) * (j / R0 + 1) * (M / (R0 * R1));
  j -= S1;
  return (j % (R0 * R1)) * (j / (R0 * R1) + 1) * (M / (R0 * R1 * R2));
}

// Radix-R stage after ns with its twiddles from a stage table (entry
// (r - 1) ns + tm); otherwise as radix_stage.
template <int N, int E, int P, int NS, int R>
__device__ __forceinline__ void radix_stage_staged(float2 (&v)[E], int p, const float2* st) {
  constexpr int U = E / R;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    float2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[u + r * U];
    const int tm = (p + P * u) & (NS - 1);
#pragma unroll
    for (int r = 1; r < R; ++r) a[r] = cmul(a[r], st[(r - 1) * NS + tm]);
    dft<R>(a);
#pragma unroll
    for (int r = 0; r < R; ++r) v[u + r * U] = a[r];
  }
}

// One FFT of length M over the tile held in v (thread (q, p) has elements
// p + P e), ending in LAST_MODE; on return v[e] is output p + P e of
// pencil q under that mapping.  The caller makes sure no thread still reads
// lds when this starts.  Twiddles from the stage table st when STAGED, else
// from the roots tw.
template <int M, class BL, int T, int SQ, int LAST_MODE, int E, int P, bool STAGED>
__device__ __forceinline__ void bluestein_fft(float2 (&v)[E], float2* lds,
                                              const float2* __restrict__ tw,
                                              const float2* st, int tid, int& q, int& p) {
  constexpr int NST = num_stages<BL>();
  constexpr int R0 = BL::R0, R1 = BL::R1, R2 = BL::R2;
  radix_stage<M, E, P, 1, R0>(v, p, tw);  // no twiddles
  if constexpr (NST == 2) {
    lds_exchange<M, E, P, T, SQ, 1, R0, LAST_MODE>(v, lds, tid, q, p);
    if constexpr (STAGED) radix_stage_staged<M, E, P, R0, R1>(v, p, st);
    else radix_stage<M, E, P, R0, R1>(v, p, tw);
  } else if constexpr (NST == 3) {
    lds_exchange<M, E, P, T, SQ, 1, R0, MODE_ROW>(v, lds, tid, q, p);
    if constexpr (STAGED) radix_stage_staged<M, E, P, R0, R1>(v, p, st);
    else radix_stage<M, E, P, R0, R1>(v, p, tw);
    __syncthreads();  // every read of the first exchange is done
    lds_exchange<M, E, P, T, SQ, R0, R1, LAST_MODE>(v, lds, tid, q, p);
    if constexpr (STAGED) radix_stage_staged<M, E, P, R0 * R1, R2>(v, p, st + (R1 - 1) * R0);
    else radix_stage<M, E, P, R0 * R1, R2>(v, p, tw);
  }
}

// Whether `entries` more float2 fit in LDS beside a tile of T pencils
// without lowering the number of workgroups a CU holds.
template <int M, int T, class BL>
constexpr bool bluestein_lds_fits(int entries) {
  constexpr int kLds = 160 * 1024, tile = T * lds_pencil_stride<M, T>() * 8;
  return num_stages<BL>() > 1 && tile + entries * 8 <= kLds &&
         kLds / (tile + entries * 8) == kLds / tile;
}
// The stage table goes to LDS where it fits; the chirp (n <= M / 2 entries,
// read again by the store) as well where both fit.
template <int M, int T, class BL>
constexpr bool bluestein_table_in_lds() {
  return bluestein_lds_fits<M, T, BL>(stage_table_size<M, BL>());
}
template <int M, int T, class BL>
constexpr bool bluestein_chirp_in_lds() {
  return bluestein_lds_fits<M, T, BL>(stage_table_size<M, BL>() + M / 2);
}
template <int M, int T, class BL>
constexpr int bluestein_lds_tables() {
  return bluestein_chirp_in_lds<M, T, BL>()
             ? stage_table_size<M, BL>() + M / 2
             : (bluestein_table_in_lds<M, T, BL>() ? stage_table_size<M, BL>() : 0);
}

// BL: register blocking of the length-m FFTs (E elements per thread).
template <int M, int T, class BL>
__global__ void __launch_bounds__(T*(M / BL::E))
bluestein_axis_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                      const float2* __restrict__ twp, const PassArgs a) {
  constexpr int E = BL::E;
  constexpr int P = M / E;
  constexpr int NST = num_stages<BL>();
  constexpr int SQ = lds_pencil_stride<M, T>();
  constexpr int LDS_ELEMS = NST > 1 ? T * SQ : 1;
  constexpr bool TWL = bluestein_table_in_lds<M, T, BL>();
  constexpr bool CHL = bluestein_chirp_in_lds<M, T, BL>();
  constexpr int ST = TWL ? stage_table_size<M, BL>() : 0;
  __shared__ float2 lds[LDS_ELEMS + bluestein_lds_tables<M, T, BL>()];
  const int64_t n = a.res_mask;
  const float2* __restrict__ chirp = twp;
  const float2* __restrict__ filt = twp + n;

  const int tid = threadIdx.x;
  // The stage twiddles go to LDS next to the tile where they fit: the later
  // radix stages of both FFTs read them, and from global memory each of
  // those stages waited on its own loads.  The first stage reads none, and
  // the first exchange's barrier orders these writes before any read.
  float2* st = lds + LDS_ELEMS;
  if constexpr (TWL) {
#pragma unroll
    for (int i = 0; i < (ST + T * P - 1) / (T * P); ++i) {
      const int j = tid + T * P * i;
      if (j < ST) st[j] = tw[stage_table_root<M, BL>(j)];
    }
  }
  // the chirp after it, for the store (the input multiply reads it from
  // global memory together with the input, before any barrier)
  float2* lchirp = st + ST;
  if constexpr (CHL) {
#pragma unroll
    for (int i = 0; i < (M / 2 + T * P - 1) / (T * P); ++i) {
      const int j = tid + T * P * i;
      if (j < n) lchirp[j] = chirp[j];
    }
  }
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  int q, p;
  thread_map<MODE_ROW, T, P>(tid, q, p);
  {
    // pencils past the end of a ragged last tile read the last pencil
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    const float2* s = src + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = p + P * e;
      float2 x = make_float2(0.f, 0.f);
      if (j < n) {
        x = s[j * a.ijs];
        if (a.conj_in) x.y = -x.y;
        x = cmul(x, chirp[j]);
      }
      v[e] = x;
    }
    bluestein_fft<M, BL, T, SQ, MODE_ROW, E, P, TWL>(v, lds, tw, st, tid, q, p);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(v[e], filt[p + P * e]);
    if constexpr (NST > 1) __syncthreads();  // the first FFT's exchanges are read
    bluestein_fft<M, BL, T, SQ, MODE_COL, E, P, TWL>(v, lds, tw, st, tid, q, p);
    const int64_t bo = tile * T + q;
    if (bo < a.B) {
      float2* d = dst + pencil_offset_any(bo, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int k = (M - (p + P * e)) & (M - 1);
        if (k < n) {
          float2 y = cmul(v[e], CHL ? lchirp[k] : chirp[k]);
          if (a.conj_out) y.y = -y.y;
          d[k * a.oks] = y;
        }
      }
    }
  }
}

template <int M, int T, class BL>
hipError_t launch_bluestein_axis(const PassArgs& a, const float2* src, float2* dst,
                                 const float2* tw, const float2* twp, hipStream_t stream) {
  constexpr int THREADS = T * (M / BL::E);
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (a.res_mask < 1 || 2 * a.res_mask - 1 > M) return hipErrorInvalidValue;
  hipLaunchKernelGGL((bluestein_axis_kernel<M, T, BL>), dim3((unsigned)blocks), dim3(THREADS),
                     0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int M, int T>
KernelInfo kernel_info_bluestein() {
  using BL = Blocking<M>;
  constexpr int E = BL::E;
  constexpr int SQ = lds_pencil_stride<M, T>();
  constexpr int LDS = (num_stages<BL>() > 1 ? T * SQ : 1) * 8 +
                      bluestein_lds_tables<M, T, BL>() * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(T * (M / E) <= 1024, "workgroup too large");
  KernelInfo k{M, T, MODE_ROW, MODE_COL, 0, T * (M / E), LDS,
               &launch_bluestein_axis<M, T, BL>, 0, 0};
  k.bluestein = 1;
  return k;
}

}  // namespace dft3d
