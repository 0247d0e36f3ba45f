// The rotate-on-write pass of length 2048 as two half-length transforms, so
// that a tile of 16 pencils fits in LDS.
//
// Splitting the index in halves (decimation in frequency, the four-step
// factorisation of eq. (3) with the radix 2 taken first):
//   a[n] = x[n] + x[n + 1024],   b[n] = (x[n] - x[n + 1024]) w_2048^n,
//   y[2k] = DFT_1024(a)[k],      y[2k + 1] = DFT_1024(b)[k].
// Each thread loads the points n and n + 1024 of its pencil, so the radix-2
// step runs in registers; the two halves then go one after the other
// through the 1024-point stages of the pass kernel (radix 32, LDS exchange,
// radix 32) in the same 16-pencil LDS tile, and each half stores its output
// rows (the even ones, then the odd ones).  A 16-pencil tile of the whole
// length would need 256 KB of LDS, and with 8 pencils the rotated store
// writes 64-byte row segments; this way every row segment is 16 pencils,
// 128 bytes.
//
// The 1024-point stage twiddles are the 2048-point roots at even indices:
// the table in LDS holds w_2048^m (m < 2048) and the radix stages are
// instantiated for length 2048, which doubles their root stride.
#pragma once

#include "pass_kernel.h"

namespace dft3d {

// Radix-2 step of the split: lo[e] = x[n] + x[n + 1024] and
// hi[e] = x[n] - x[n + 1024] for n = p + P e; the twiddle w^n of the
// differences is applied when their half starts (halves_half), so that its
// table entries are not held in registers during the first half.
template <int E, bool MV>
__device__ __forceinline__ void halves_split(float2 (&lo)[E], float2 (&hi)[E]) {
  if constexpr (MV) return;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const float2 u = lo[e], w = hi[e];
    lo[e] = make_float2(u.x + w.x, u.y + w.y);
    hi[e] = make_float2(u.x - w.x, u.y - w.y);
  }
}

// The second radix-32 stage of a half (after 32, thread p owns butterfly
// t = p), its twiddles w_1024^{p r} = w_2048^{2 p r} formed as the products
// w_2048^{16 p k} w_2048^{2 p j} (r = 8 k + j) of ten table entries: the 31
// entries the stage would otherwise read stay out of the registers, which
// the other half's 32 points share with it.
template <int P, bool MV>
__device__ __forceinline__ void halves_stage2(float2 (&v)[32], int p, const float2* roots) {
  if constexpr (MV) return;
  float2 lo[8], hi[4];
#pragma unroll
  for (int j = 1; j < 8; ++j) lo[j] = roots[2 * p * j];
#pragma unroll
  for (int k = 1; k < 4; ++k) hi[k] = roots[16 * p * k];
#pragma unroll
  for (int r = 1; r < 32; ++r) {
    const int j = r & 7, k = r >> 3;
    const float2 w = k == 0 ? lo[j] : (j == 0 ? hi[k] : cmul(hi[k], lo[j]));
    v[r] = cmul(v[r], w);
  }
  dft<32>(v);
}

// One half (H = 0: the sums a, H = 1: the twiddled differences b) of a
// tile through the 1024-point stages, stored at the output rows 2k + H.
// SYNC: wait before the exchange writes LDS (a previous exchange's reads).
template <int T, int NT, int SQ, int H, bool SYNC>
__device__ __forceinline__ void halves_half(float2 (&v)[32], float2* dst, const float2* roots,
                                            float2* lds, const PassArgs& a, int64_t tile,
                                            int tid) {
  constexpr int E = 32, P = 32;
  constexpr bool MV = move_only(NT);
  int q, p;
  thread_map<MODE_ROW, T, P>(tid, q, p);
  if constexpr (H == 1 && !MV) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(v[e], roots[p + P * e]);
  }
  radix_stage<2048, E, P, 1, 32, MV>(v, p, roots);
  if constexpr (SYNC) __syncthreads();
  lds_exchange<1024, E, P, T, SQ, 1, 32, MODE_COL>(v, lds, tid, q, p);
  halves_stage2<P, MV>(v, p, roots);
  const int64_t b = tile * T + q;
  if (b < a.B) {
    float2* d = dst + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    d += (int64_t)(2 * p + H) * a.oks;              // output row 2 (p + P e) + H
    const int64_t step = (int64_t)(2 * P) * a.oks;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 w = v[e];
      if (a.conj_out) w.y = -w.y;
      store_c64(d + e * step, w, nt_stores(NT));
    }
  }
}

// Conjugation of an inverse transform's input and the radix-2 split.
template <int NT>
__device__ __forceinline__ void halves_begin(float2 (&lo)[32], float2 (&hi)[32],
                                             const PassArgs& a) {
  if (a.conj_in) {
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      lo[e].y = -lo[e].y;
      hi[e].y = -hi[e].y;
    }
  }
  halves_split<32, move_only(NT)>(lo, hi);
}

// Loads of one tile: thread (q, p) of the load mapping gets the points
// p + P e (lo) and 1024 + p + P e (hi) of pencil q; pencils past the end of
// a ragged last tile read the last pencil (in bounds, never stored).
template <int T, int NT>
__device__ __forceinline__ void halves_load(float2 (&lo)[32], float2 (&hi)[32], const float2* src,
                                            const PassArgs& a, int64_t tile, int tid,
                                            bool low, bool high) {
  constexpr int P = 32;
  int q, p;
  thread_map<MODE_ROW, T, P>(tid, q, p);
  int64_t b = tile * T + q;
  b = b < a.B ? b : a.B - 1;
  const float2* s = src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2) + p;
  if (low) {
#pragma unroll
    for (int e = 0; e < 32; ++e) lo[e] = load_c64(s + P * e, nt_loads(NT));
  }
  if (high) {
#pragma unroll
    for (int e = 0; e < 32; ++e) hi[e] = load_c64(s + 1024 + P * e, nt_loads(NT));
  }
}

// One workgroup per tile.
template <int T, int NT>
__global__ void __launch_bounds__(T * 32)
fft_pass_halves(const float2* src, float2* dst, const float2* __restrict__ tw,
                const float2* __restrict__ twp, const PassArgs a) {
  constexpr int SQ = lds_pencil_stride<1024, T>();
  __shared__ float2 lds[T * SQ];
  __shared__ float2 roots[2048];
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  float2 lo[32], hi[32];
  halves_load<T, NT>(lo, hi, src, a, tile, tid, true, true);
  for (int i = tid; i < 2048; i += T * 32) roots[i] = tw[i];
  __syncthreads();
  halves_begin<NT>(lo, hi, a);
  halves_half<T, NT, SQ, 0, false>(lo, dst, roots, lds, a, tile, tid);
  halves_half<T, NT, SQ, 1, true>(hi, dst, roots, lds, a, tile, tid);
}

template <int T, int NT>
hipError_t launch_halves(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                         const float2* twp, hipStream_t stream) {
  const int64_t tiles = (a.B + T - 1) / T;
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_pass_halves<T, NT>), dim3((unsigned)tiles), dim3(T * 32), 0, stream,
                     src, dst, tw, twp, a);
  return hipGetLastError();
}

// One tile per workgroup only: the LDS tile allows one resident workgroup
// per CU, and a persistent form that loads the next tile's lower halves
// during the upper halves' stages needs more registers than its two waves
// per SIMD have (it spilled and measured slower).
template <int T, int NT>
KernelInfo kernel_info_halves() {
  constexpr int LDS = (T * lds_pencil_stride<1024, T>() + 2048) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(T * 32 <= 1024, "workgroup too large");
  KernelInfo k{2048, T, MODE_ROW, MODE_COL, 0, T * 32, LDS, &launch_halves<T, NT>, 0, NT & 3};
  k.move_only = move_only(NT) ? 1 : 0;
  k.r0 = 2;
  k.r1 = 32;
  k.r2 = 32;
  k.halves = 1;
  return k;
}

}  // namespace dft3d
