// A pass of length N as two half-length transforms, so that a tile of twice
// as many pencils fits in LDS: the rotate-on-write pass of length 2048 in
// 16-pencil tiles and the strided (column) pass of length 1024 in 32-pencil
// tiles.
//
// Splitting the index in halves (decimation in frequency, the four-step
// factorisation of eq. (3) with the radix 2 taken first), with M = N / 2:
//   a[n] = x[n] + x[n + M],   b[n] = (x[n] - x[n + M]) w_N^n,
//   y[2k] = DFT_M(a)[k],      y[2k + 1] = DFT_M(b)[k].
// Each thread loads the points n and n + M of its pencil, so the radix-2
// step runs in registers; the two halves then go one after the other
// through the two M-point stages of the pass kernel (radix R0, LDS
// exchange, radix R1) in the same LDS tile, and each half stores its output
// rows (the even ones, then the odd ones).  A tile of the whole length
// would need twice the LDS: with the split, the stored (and, for strided
// loads, the loaded) row segments are T pencils long, 128 bytes at
// N = 2048 and 256 bytes at N = 1024, where the whole-length kernels take
// 8 and 16 pencils.
//
// The M-point stage twiddles are the N-point roots at even indices: the
// table in LDS holds w_N^m (m < N).
#pragma once

#include "pass_kernel.h"

namespace dft3d {

// Radix-2 step of the split: lo[e] = x[n] + x[n + M] and
// hi[e] = x[n] - x[n + M] for n = p + P e; the twiddle w^n of the
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

// The second stage of a half (radix R after NS = M / R; thread p runs the
// butterflies t = p + P u), its twiddles w_M^{t r} = w_N^{2 t r} formed as
// the products w_N^{16 t k} w_N^{2 t j} (r = 8 k + j) of a few table
// entries: the R - 1 entries a butterfly would otherwise read stay out of
// the registers, which the other half's points share with it.
template <int N, int E, int P, int NS, int R, bool MV>
__device__ __forceinline__ void halves_stage2(float2 (&v)[E], int p, const float2* roots) {
  if constexpr (MV) return;
  static_assert(R % 8 == 0 && NS * R == N / 2, "second stage of a half");
  constexpr int U = E / R;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = (p + P * u) & (NS - 1);
    float2 lo[8], hi[R / 8];
#pragma unroll
    for (int j = 1; j < 8; ++j) lo[j] = roots[2 * t * j];
#pragma unroll
    for (int k = 1; k < R / 8; ++k) hi[k] = roots[16 * t * k];
    float2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[u + r * U];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const int j = r & 7, k = r >> 3;
      const float2 w = k == 0 ? lo[j] : (j == 0 ? hi[k] : cmul(hi[k], lo[j]));
      a[r] = cmul(a[r], w);
    }
    dft<R>(a);
#pragma unroll
    for (int r = 0; r < R; ++r) v[u + r * U] = a[r];
  }
}

// One half (H = 0: the sums a, H = 1: the twiddled differences b) of a
// tile through the M-point stages, stored at the output rows 2k + H.
// Half 0 parks the other half (`other`, load mapping) in the LDS tile while
// its second stage runs and half 1 takes it back: the LDS tile is free once
// the exchange has been read, and the other half's registers would
// otherwise be live at the peak of the second stage (the kernel spilled
// there, and the spills cost HBM traffic).  Every thread takes back what it
// parked itself; the barriers keep the exchanges of the other threads away.
template <int N, int T, int LM, int SM, int NT, int SQ, int H, bool SYNC0 = false>
__device__ __forceinline__ void halves_half(float2 (&v)[32], float2 (&other)[32], float2* dst,
                                            const float2* roots, float2* lds,
                                            const PassArgs& a, int64_t tile, int tid) {
  using BL = Blocking<N / 2>;
  constexpr int E = 32, P = N / 2 / E;
  static_assert(BL::E == E && num_stages<BL>() == 2, "two-stage halves of 32 per thread");
  constexpr bool MV = move_only(NT);
  int ql, pl;  // the load mapping: where the parked half lives
  thread_map<LM, T, P>(tid, ql, pl);
  float2* mine = lds + ql * SQ;
  if constexpr (H == 1) {
    __syncthreads();  // no values of the parked half stay in registers
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = mine[lds_pad_index(pl + P * e)];
    if constexpr (!MV) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(v[e], roots[pl + P * e]);
    }
  }
  radix_stage<N, E, P, 1, BL::R0, MV>(v, pl, roots);
  // H = 1: every parked point is taken back; SYNC0: the previous tile's
  // exchange reads are done
  if constexpr (H == 1 || SYNC0) __syncthreads();
  int q = ql, p = pl;
  lds_exchange<N / 2, E, P, T, SQ, 1, BL::R0, SM>(v, lds, tid, q, p);
  if constexpr (H == 0) {
    __syncthreads();  // every exchange read is done: park the other half
#pragma unroll
    for (int e = 0; e < E; ++e) mine[lds_pad_index(pl + P * e)] = other[e];
  }
  halves_stage2<N, E, P, BL::R0, BL::R1, MV>(v, p, roots);
  const int64_t b = tile * T + q;
  if (b < a.B) {
    float2* d = dst + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    const int64_t os = SM == MODE_ROW ? 1 : a.oks;
    d += (int64_t)(2 * p + H) * os;                 // output row 2 (p + P e) + H
    const int64_t step = (int64_t)(2 * P) * os;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 w = v[e];
      if (a.conj_out) w.y = -w.y;
      store_c64(d + e * step, w, nt_stores(NT));
    }
  }
}

// Loads of one tile: thread (q, p) of the load mapping gets the points
// p + P e (lo) and M + p + P e (hi) of pencil q; pencils past the end of a
// ragged last tile read the last pencil (in bounds, never stored).
template <int N, int T, int LM, int NT>
__device__ __forceinline__ void halves_load(float2 (&lo)[32], float2 (&hi)[32], const float2* src,
                                            const PassArgs& a, int64_t tile, int tid,
                                            bool low = true, bool high = true) {
  constexpr int P = N / 2 / 32;
  int q, p;
  thread_map<LM, T, P>(tid, q, p);
  int64_t b = tile * T + q;
  b = b < a.B ? b : a.B - 1;
  const float2* s = src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
  const int64_t is = LM == MODE_ROW ? 1 : a.ijs;
  s += (int64_t)p * is;
  if (low) {
#pragma unroll
    for (int e = 0; e < 32; ++e) lo[e] = load_c64(s + (int64_t)(P * e) * is, nt_loads(NT));
  }
  if (high) {
#pragma unroll
    for (int e = 0; e < 32; ++e)
      hi[e] = load_c64(s + (int64_t)(N / 2 + P * e) * is, nt_loads(NT));
  }
}

// One workgroup per tile.  In place (src == dst, COL to COL) is allowed:
// the whole tile is in registers before its first store, and tiles are
// disjoint.
template <int N, int T, int LM, int SM, int NT>
__global__ void __launch_bounds__(T * (N / 64))
fft_pass_halves(const float2* src, float2* dst, const float2* __restrict__ tw,
                const float2* __restrict__ twp, const PassArgs a) {
  constexpr int SQ = lds_pencil_stride<N / 2, T>();
  __shared__ float2 lds[T * SQ];
  __shared__ float2 roots[N];
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  float2 lo[32], hi[32];
  halves_load<N, T, LM, NT>(lo, hi, src, a, tile, tid);
  for (int i = tid; i < N; i += T * (N / 64)) roots[i] = tw[i];
  __syncthreads();
  if (a.conj_in) {  // inverse as conj(DFT(conj(x)))
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      lo[e].y = -lo[e].y;
      hi[e].y = -hi[e].y;
    }
  }
  halves_split<32, move_only(NT)>(lo, hi);
  halves_half<N, T, LM, SM, NT, SQ, 0>(lo, hi, dst, roots, lds, a, tile, tid);
  halves_half<N, T, LM, SM, NT, SQ, 1>(hi, lo, dst, roots, lds, a, tile, tid);
}

// Persistent form: about one resident workgroup per CU walks the tiles
// (w, w + G, ...); once the first half is stored and the second parked in
// LDS, both halves of the next tile are loaded into the freed registers
// while the second half goes through its stages.
template <int N, int T, int LM, int SM, int NT>
__global__ void __launch_bounds__(T * (N / 64))
fft_pass_halves_persistent(const float2* src, float2* dst, const float2* __restrict__ tw,
                           const float2* __restrict__ twp, const PassArgs a) {
  constexpr int SQ = lds_pencil_stride<N / 2, T>();
  __shared__ float2 lds[T * SQ];
  __shared__ float2 roots[N];
  const int tid = threadIdx.x;
  const int64_t ntiles = (a.B + T - 1) / T;
  const int64_t G = gridDim.x;
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  const int64_t last = ntiles - 1;
  float2 lo[32], hi[32];
  halves_load<N, T, LM, NT>(lo, hi, src, a, tile_index(w, ntiles, a.xcd_remap), tid);
  for (int i = tid; i < N; i += T * (N / 64)) roots[i] = tw[i];
  __syncthreads();
  while (true) {
    const int64_t tile = tile_index(w, ntiles, a.xcd_remap);
    if (a.conj_in) {
#pragma unroll
      for (int e = 0; e < 32; ++e) {
        lo[e].y = -lo[e].y;
        hi[e].y = -hi[e].y;
      }
    }
    halves_split<32, move_only(NT)>(lo, hi);
    halves_half<N, T, LM, SM, NT, SQ, 0, true>(lo, hi, dst, roots, lds, a, tile, tid);
    const int64_t wn = w + G;
    const int64_t next = tile_index(wn < last ? wn : last, ntiles, a.xcd_remap);
    // the lower halves of the next tile (past the last tile: the last again)
    halves_load<N, T, LM, NT>(lo, hi, src, a, next, tid, true, false);
    halves_half<N, T, LM, SM, NT, SQ, 1>(hi, hi, dst, roots, lds, a, tile, tid);
    w = wn;
    if (w >= ntiles) break;
    halves_load<N, T, LM, NT>(lo, hi, src, a, next, tid, false, true);
  }
}

template <int N, int T, int LM, int SM, int NT>
hipError_t launch_halves_persistent(const PassArgs& a, const float2* src, float2* dst,
                                    const float2* tw, const float2* twp, hipStream_t stream) {
  const int64_t tiles = (a.B + T - 1) / T;
  if (tiles <= 0) return hipSuccess;
  static int per_cu = -1;  // resident workgroups per CU for this kernel
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fft_pass_halves_persistent<N, T, LM, SM, NT>, T * (N / 64), 0) != hipSuccess)
      return hipGetLastError();
    per_cu = nb > 0 ? nb : 1;
  }
  int64_t grid = (int64_t)device_cu_count() * per_cu;
  if (grid > tiles) grid = tiles;
  hipLaunchKernelGGL((fft_pass_halves_persistent<N, T, LM, SM, NT>), dim3((unsigned)grid),
                     dim3(T * (N / 64)), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int N, int T, int LM, int SM, int NT>
hipError_t launch_halves(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                         const float2* twp, hipStream_t stream) {
  const int64_t tiles = (a.B + T - 1) / T;
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_pass_halves<N, T, LM, SM, NT>), dim3((unsigned)tiles),
                     dim3(T * (N / 64)), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

// The LDS tile allows one resident workgroup per CU: the one-tile form
// leaves the memory system idle while a workgroup computes, the persistent
// form overlaps the next tile's lower halves with the current second half.
template <int N, int T, int LM, int SM, int NT>
KernelInfo kernel_info_halves() {
  constexpr int LDS = (T * lds_pencil_stride<N / 2, T>() + N) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(T * (N / 64) <= 1024, "workgroup too large");
  KernelInfo k{N, T, LM, SM, 0, T * (N / 64), LDS, &launch_halves<N, T, LM, SM, NT>, 0, NT & 3};
  k.move_only = move_only(NT) ? 1 : 0;
  k.r0 = 2;
  k.r1 = Blocking<N / 2>::R0;
  k.r2 = Blocking<N / 2>::R1;
  k.halves = 1;
  return k;
}

template <int N, int T, int LM, int SM, int NT>
KernelInfo kernel_info_halves_persistent() {
  KernelInfo k = kernel_info_halves<N, T, LM, SM, NT>();
  k.launch = &launch_halves_persistent<N, T, LM, SM, NT>;
  k.persistent = 1;
  return k;
}

// Ordinary and streaming accesses, and their move-only twins; with PERS the
// persistent forms too.
template <int N, int T, int LM, int SM, bool PERS>
void add_halves_kernels(std::vector<KernelInfo>& v) {
  if constexpr (PERS) {
    v.push_back(kernel_info_halves_persistent<N, T, LM, SM, 0>());
    v.push_back(kernel_info_halves_persistent<N, T, LM, SM, 1>());
    v.push_back(kernel_info_halves_persistent<N, T, LM, SM, 4>());
    v.push_back(kernel_info_halves_persistent<N, T, LM, SM, 5>());
  }
  v.push_back(kernel_info_halves<N, T, LM, SM, 0>());
  v.push_back(kernel_info_halves<N, T, LM, SM, 1>());
  v.push_back(kernel_info_halves<N, T, LM, SM, 4>());
  v.push_back(kernel_info_halves<N, T, LM, SM, 5>());
}

}  // namespace dft3d
