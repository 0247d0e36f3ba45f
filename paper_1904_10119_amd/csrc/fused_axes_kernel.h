// Volumetric schedule: the second half of one axis and the first half of the
// next in one pass (Fig. 9, eqs. (13)-(17) applied to two axes at once).
//
// Axis d of length n_d = a * b is split four-step style; its first half V1
// has left T0 at axis position k a + l (k < b, l < a).  The fused pass
// finishes axis d -- DFT_a over l, natural output k + b l' -- and starts
// axis d-1 (length n' = A' B', A' = B' = a): for residue r' of axis d-1,
// DFT_a over m of the rows r' + A' m, times w_{n'}^{r' k2}, stored at row
// r' + A' k2.  A workgroup owns one residue r', all a rows, and KC
// consecutive V2 runs (CONTIG: runs contiguous along axis d, the innermost
// axis) or one run and KC consecutive innermost points (runs strided), so
// both the loads and the stores move KC * 8-byte segments or longer.
//
// Stage 1: thread = one run (c, kk, m) -> DFT_a in registers -> LDS tile
// [m][j], j = c + C (kk + K l').  Stage 2: thread = one column j -> the a
// rows from LDS -> DFT_a -> twiddle -> store.
//
// SHUF = 1 (the shuffled layout, Section 2.4): axis d's final exchange is
// left out, so output l' of run k' stays where its input run lay, at axis
// position a k' + l' (the pass's run field has equal input and output
// strides); axis d-1 is written as in natural order.
//
// PassArgs fields used: tile t splits into f0 = t & m0, f1 = (t >> s0) & m1
// (the residue r'), f2 = t >> s1; tile bases f0 is0 + f1 is1 + f2 is2 (in)
// and f0 os0 + f1 os1 + f2 os2 (out); ijs = row step A' * S_{d-1}; oks =
// S_d (axis d stride); res_mask = b; twp_mask = n' - 1.
//
// SHUF = 3 (fused_axes = 3), the inverse from the shuffled order: the
// transpose of the SHUF = 1 pass (every DFT matrix and twiddle diagonal is
// symmetric, so the transpose of a product of passes runs the passes'
// transposes in reverse order).  Axis d-1 has had its first half and gets
// its second (DFT over the rows m, no twiddle); run k' of axis d
// (positions a k' + l', contiguous in the shuffled order) gets its first
// half: DFT_a over l', times w_{n_d}^{k' a'}, in place at a k' + a'.  The
// two act on different axes and commute, so the tile runs in the SHUF = 1
// order and layout (runs first, then rows) with the twiddle moved to stage 1;
// twp is axis d's table, twp_mask = n_d - 1, and the run index k' is
// f0 KC + kk (CONTIG) or f2 (runs strided).  With res_shift = 1 the pass
// also owes axis d-1's first-half twiddle (its first half ran as a pass
// without it): the rows get w_{n_{d-1}}^{r' m} before their DFT, from tw
// (axis d-1's table), res_mask = n_{d-1} - 1.
#pragma once

#include "pass_kernel.h"

namespace dft3d {

template <int A, int KC> constexpr int fused_row() { return KC * A + ((KC * A) >> 5) + 1; }

// SHUF = 3 with contiguous runs: the tile's KC runs have KC different run
// indices k', so the stage-1 twiddles w_{n_d}^{k' l'} would be a KC-way
// gather per element; the workgroup reads the KC x A block once (one entry
// per thread) into LDS rows of A + 1 entries.
template <int A, int KC, int CONTIG, int SHUF>
constexpr int fused_tw_lds() { return SHUF == 3 && CONTIG ? KC * (A + 1) : 1; }

template <int A, int KC, int CONTIG, int SHUF>
__device__ __forceinline__ void fused_tw_block(float2* twl, const float2* __restrict__ twp,
                                               const PassArgs& a, int64_t f0, int tid) {
  if (SHUF == 3 && CONTIG) {
    const int kk = tid / A, lp = tid % A;  // A * KC threads: one entry each
    twl[kk * (A + 1) + lp] = twp[((f0 * KC + kk) * lp) & a.twp_mask];
  }
}

struct FusedTile {
  int64_t in_base, out_base, r;  // tile bases and the residue r' of axis d-1
  int64_t f0, f2;                // the other two tile fields
};

__device__ __forceinline__ FusedTile fused_tile(int64_t t, const PassArgs& a) {
  const int64_t f0 = t & a.m0, f1 = (t >> a.s0) & a.m1, f2 = t >> a.s1;
  return FusedTile{f0 * a.is0 + f1 * a.is1 + f2 * a.is2, f0 * a.os0 + f1 * a.os1 + f2 * a.os2,
                   f1, f0, f2};
}

// Stage-1 inputs of this thread's run (c, kk, m): elements l along axis d.
template <int A, int KC, int CONTIG>
__device__ __forceinline__ void fused_load(float2 (&v)[A], const float2* src, const PassArgs& a,
                                           const FusedTile& ft, int tid) {
  constexpr int K = CONTIG ? KC : 1;
  constexpr int C = CONTIG ? 1 : KC;
  const int c = tid % C, kk = (tid / C) % K, m = tid / KC;
  const float2* s = src + ft.in_base + m * a.ijs + (int64_t)(kk * A) * a.oks + c;
#pragma unroll
  for (int l = 0; l < A; ++l) v[l] = s[l * a.oks];
}

// Column j of the LDS tile holding output l' of run (c, kk): natural order
// runs kk fastest after c (a stage-2 wave then stores consecutive kk, which
// are consecutive along axis d); the shuffled order runs l' fastest after c
// (consecutive l' are consecutive along axis d there).
template <int A, int KC, int CONTIG, int SHUF>
__device__ __forceinline__ int fused_column(int c, int kk, int lp) {
  constexpr int K = CONTIG ? KC : 1;
  constexpr int C = CONTIG ? 1 : KC;
  return SHUF ? c + C * (lp + A * kk) : c + C * (kk + K * lp);  // SHUF 1 or 3
}

// Stage 1: DFT_a over l in registers (SHUF = 3: times w_{n_d}^{k' l'}),
// results to the LDS tile [m][j].
template <int A, int KC, int CONTIG, int SHUF>
__device__ __forceinline__ void fused_stage1(float2 (&v)[A], float2* lds, const float2* twl,
                                             const float2* __restrict__ twp, const PassArgs& a,
                                             const FusedTile& ft, int tid) {
  constexpr int K = CONTIG ? KC : 1;
  constexpr int C = CONTIG ? 1 : KC;
  const int c = tid % C, kk = (tid / C) % K, m = tid / KC;
  if (a.conj_in) {
#pragma unroll
    for (int l = 0; l < A; ++l) v[l].y = -v[l].y;
  }
  dft<A>(v);
  if (SHUF == 3 && CONTIG) {  // run index k' = f0 KC + kk: the LDS block
#pragma unroll
    for (int lp = 1; lp < A; ++lp) v[lp] = cmul(v[lp], twl[kk * (A + 1) + lp]);
  } else if (SHUF == 3) {  // k' = f2, one per tile
#pragma unroll
    for (int lp = 1; lp < A; ++lp) v[lp] = cmul(v[lp], twp[(ft.f2 * lp) & a.twp_mask]);
  }
  float2* row = lds + m * fused_row<A, KC>();
#pragma unroll
  for (int lp = 0; lp < A; ++lp)
    row[lds_pad_index(fused_column<A, KC, CONTIG, SHUF>(c, kk, lp))] = v[lp];
}

// Stage 2: column j = tid over the a rows, DFT, twiddle w_{n'}^{r' k2}
// (SHUF = 3: none after, w_{n_{d-1}}^{r' m} before if owed), store.
template <int A, int KC, int CONTIG, int SHUF>
__device__ __forceinline__ void fused_stage2(const float2* lds, float2* dst,
                                             const float2* __restrict__ tw,
                                             const float2* __restrict__ twp, const PassArgs& a,
                                             const FusedTile& ft, int tid) {
  constexpr int K = CONTIG ? KC : 1;
  constexpr int C = CONTIG ? 1 : KC;
  float2 v[A];
#pragma unroll
  for (int m = 0; m < A; ++m) v[m] = lds[m * fused_row<A, KC>() + lds_pad_index(tid)];
  if (SHUF == 3 && a.res_shift) {
#pragma unroll
    for (int m = 1; m < A; ++m) v[m] = cmul(v[m], tw[(ft.r * m) & a.res_mask]);
  }
  dft<A>(v);
  // column tid's run and output (the inverse of fused_column)
  const int c = tid % C;
  const int kk = SHUF ? tid / (C * A) : (tid / C) % K;
  const int lp = SHUF ? (tid / C) % A : tid / KC;
  const int64_t pos = SHUF ? (int64_t)kk * A + lp : kk + a.res_mask * lp;
  float2* d = dst + ft.out_base + pos * a.oks + c;
#pragma unroll
  for (int k2 = 0; k2 < A; ++k2) {
    float2 w = SHUF == 3 ? v[k2] : cmul(v[k2], twp[(ft.r * k2) & a.twp_mask]);
    if (a.conj_out) w.y = -w.y;
    d[k2 * a.ijs] = w;
  }
}

// One tile per workgroup.
template <int A, int KC, int CONTIG, int SHUF>
__global__ void __launch_bounds__(A* KC)
fft_fused_axes_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                      const float2* __restrict__ twp, const PassArgs a) {
  __shared__ float2 lds[A * fused_row<A, KC>()];
  __shared__ float2 twl[fused_tw_lds<A, KC, CONTIG, SHUF>()];
  const int tid = threadIdx.x;
  const FusedTile ft = fused_tile(blockIdx.x, a);
  float2 v[A];
  fused_load<A, KC, CONTIG>(v, src, a, ft, tid);
  if (SHUF == 3 && CONTIG) {
    fused_tw_block<A, KC, CONTIG, SHUF>(twl, twp, a, ft.f0, tid);
    __syncthreads();
  }
  fused_stage1<A, KC, CONTIG, SHUF>(v, lds, twl, twp, a, ft, tid);
  __syncthreads();
  fused_stage2<A, KC, CONTIG, SHUF>(lds, dst, tw, twp, a, ft, tid);
}

// Persistent form: about one workgroup per CU walks the tiles w, w + G, ...
// and loads the next tile's runs into registers as soon as the current
// tile's first stage has left them, so the loads are in flight during the
// second stage and the stores.  Past the last tile the prefetch re-reads
// the last tile (in bounds).
template <int A, int KC, int CONTIG, int SHUF>
__global__ void __launch_bounds__(A* KC)
fft_fused_axes_persistent(const float2* src, float2* dst, const float2* __restrict__ tw,
                          const float2* __restrict__ twp, const PassArgs a) {
  __shared__ float2 lds[A * fused_row<A, KC>()];
  __shared__ float2 twl[fused_tw_lds<A, KC, CONTIG, SHUF>()];
  const int tid = threadIdx.x;
  const int64_t ntiles = a.B, G = gridDim.x, last = ntiles - 1;
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  float2 v[A];
  fused_load<A, KC, CONTIG>(v, src, a, fused_tile(w, a), tid);
  while (true) {
    const FusedTile ft = fused_tile(w, a);
    if (SHUF == 3 && CONTIG) {  // the previous tile's stage 1 is past a barrier
      fused_tw_block<A, KC, CONTIG, SHUF>(twl, twp, a, ft.f0, tid);
      __syncthreads();
    }
    fused_stage1<A, KC, CONTIG, SHUF>(v, lds, twl, twp, a, ft, tid);
    __syncthreads();
    const int64_t wn = w + G;
    fused_load<A, KC, CONTIG>(v, src, a, fused_tile(wn < last ? wn : last, a), tid);
    fused_stage2<A, KC, CONTIG, SHUF>(lds, dst, tw, twp, a, ft, tid);
    __syncthreads();  // every read of the tile is done before the next writes
    w = wn;
    if (w >= ntiles) break;
  }
}

template <int A, int KC, int CONTIG, int SHUF>
hipError_t launch_fused_axes(const PassArgs& a, const float2* src, float2* dst,
                             const float2* tw, const float2* twp, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  if (a.B > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_fused_axes_kernel<A, KC, CONTIG, SHUF>), dim3((unsigned)a.B),
                     dim3(A * KC), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

int device_cu_count();

template <int A, int KC, int CONTIG, int SHUF>
hipError_t launch_fused_axes_persistent(const PassArgs& a, const float2* src, float2* dst,
                                        const float2* tw, const float2* twp,
                                        hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  static int per_cu = -1;  // resident workgroups per CU for this kernel
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fft_fused_axes_persistent<A, KC, CONTIG, SHUF>, A * KC, 0) != hipSuccess)
      return hipGetLastError();
    per_cu = nb > 0 ? nb : 1;
  }
  int64_t grid = (int64_t)device_cu_count() * per_cu;
  if (grid > a.B) grid = a.B;
  hipLaunchKernelGGL((fft_fused_axes_persistent<A, KC, CONTIG, SHUF>), dim3((unsigned)grid),
                     dim3(A * KC), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int A, int KC, int CONTIG, int PERS, int SHUF = 0>
KernelInfo kernel_info_fused_axes() {
  constexpr int LDS = (A * fused_row<A, KC>() + fused_tw_lds<A, KC, CONTIG, SHUF>()) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(A * KC <= 1024, "workgroup too large");
  const int mode = CONTIG ? MODE_ROW : MODE_COL;
  KernelInfo k{A, KC, mode, mode, 1, A * KC, LDS,
               PERS ? &launch_fused_axes_persistent<A, KC, CONTIG, SHUF>
                    : &launch_fused_axes<A, KC, CONTIG, SHUF>,
               PERS, 0, 0};
  k.fused_axes = SHUF == 3 ? 3 : (SHUF ? 2 : 1);
  return k;
}

}  // namespace dft3d
