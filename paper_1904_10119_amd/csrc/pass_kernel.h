// The batched 1D FFT pass kernel (Stockham, radix 2..32 in registers, LDS
// exchanges between radix stages) with configurable load and store layouts.
//
// One workgroup transforms a tile of T pencils of length N.  Thread p of a
// pencil (0 <= p < P = N / E) holds the E elements p + P e in registers
// before the first stage and, after the last stage, the E outputs p + P e.
// Radix stage s (radix R, Ns = product of the earlier radices) runs the E/R
// butterflies t = p + P u of that thread:
//   a_r = v[u + r E/R] * w_{Ns R}^{(t mod Ns) r},   a = DFT_R(a),
// and output r of butterfly t belongs at position
//   (t div Ns) Ns R + (t mod Ns) + r Ns,
// which is where the next stage's thread picks it up through LDS.  This is
// the four-step factorisation of eq. (3) applied recursively (stage I = the
// butterflies, stage II = the twiddle, stage III = the LDS exchange).
//
// The layout change between the 3D passes (the ROTE pack / all-to-all /
// unpack of Section 3.1.3, Fig. 8) is folded into the loads and stores: the
// thread-to-(pencil, element) mapping before the first stage follows the
// load mode and the mapping after the last exchange follows the store mode,
// so both sides touch memory in segments of at least 128 bytes whenever the
// tile allows it.
#pragma once

#include "fft_device.h"
#include "internal.h"

namespace dft3d {

// Register blocking per transform length: E elements per thread and up to
// three radix stages (1 = unused).
template <int N> struct Blocking;
#define DFT3D_BLOCKING(N_, E_, R0_, R1_, R2_)                               \
  template <> struct Blocking<N_> {                                         \
    static constexpr int E = E_, R0 = R0_, R1 = R1_, R2 = R2_;              \
  };
DFT3D_BLOCKING(1, 1, 1, 1, 1)
DFT3D_BLOCKING(2, 2, 2, 1, 1)
DFT3D_BLOCKING(4, 4, 4, 1, 1)
DFT3D_BLOCKING(8, 8, 8, 1, 1)
DFT3D_BLOCKING(16, 16, 16, 1, 1)
DFT3D_BLOCKING(32, 32, 32, 1, 1)
DFT3D_BLOCKING(64, 8, 8, 8, 1)
DFT3D_BLOCKING(128, 16, 16, 8, 1)
DFT3D_BLOCKING(256, 16, 16, 16, 1)
DFT3D_BLOCKING(512, 32, 32, 16, 1)
DFT3D_BLOCKING(1024, 32, 32, 32, 1)
DFT3D_BLOCKING(2048, 32, 32, 8, 8)
DFT3D_BLOCKING(4096, 32, 32, 16, 8)
#undef DFT3D_BLOCKING

template <int N> constexpr int num_stages() {
  return Blocking<N>::R1 == 1 ? 1 : (Blocking<N>::R2 == 1 ? 2 : 3);
}

// LDS: pencil-major, one pad element per 32 so that the stride-R writes of
// the first stage spread over all banks, and a pencil stride chosen so that
// a wavefront reading one element row across the tile (store mode COL:
// T pencils x 64/T threads) covers every bank pair at most twice.
__host__ __device__ constexpr int lds_pad_index(int i) { return i + (i >> 5); }
template <int N, int T> constexpr int lds_pencil_stride() {
  int base = N + (N >> 5);
  int want = (T >= 64) ? 1 : ((64 / T) & 31);
  int s = base;
  while ((s & 31) != want) ++s;
  return s;
}

template <int MODE, int T, int P>
__device__ __forceinline__ void thread_map(int tid, int& q, int& p) {
  if constexpr (MODE == MODE_ROW) {
    q = tid / P;
    p = tid % P;
  } else {
    q = tid % T;
    p = tid / T;
  }
}

__device__ __forceinline__ int64_t pencil_offset(int64_t b, int64_t m0, int64_t m1,
                                                 int s0, int s1, int64_t st0,
                                                 int64_t st1, int64_t st2) {
  return (b >> s1) * st2 + ((b >> s0) & m1) * st1 + (b & m0) * st0;
}

// Consecutive tiles land on one XCD: workgroups are dispatched round-robin
// over the 8 XCDs, so workgroup w runs on XCD w % 8.
__device__ __forceinline__ int64_t tile_index(int64_t bid, int64_t nb, int remap) {
  if (!remap) return bid;
  const int64_t full = nb & ~int64_t(7);
  if (bid >= full) return bid;
  return (bid & 7) * (full >> 3) + (bid >> 3);
}

template <int N, int E, int P, int NS, int R>
__device__ __forceinline__ void radix_stage(float2 (&v)[E], int p,
                                            const float2* __restrict__ tw) {
  constexpr int U = E / R;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    float2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[u + r * U];
    if constexpr (NS > 1) {
      const int tm = (p + P * u) & (NS - 1);
      constexpr int STEP = N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) a[r] = cmul(a[r], tw[tm * r * STEP]);
    }
    dft<R>(a);
#pragma unroll
    for (int r = 0; r < R; ++r) v[u + r * U] = a[r];
  }
}

// Write the outputs of a stage (radix R after NS) to LDS at their Stockham
// positions, then read back the elements p + P e under the next mapping.
template <int N, int E, int P, int T, int SQ, int NS, int R, int NEXT_MODE>
__device__ __forceinline__ void lds_exchange(float2 (&v)[E], float2* lds, int tid,
                                             int& q, int& p) {
  constexpr int U = E / R;
  float2* mine = lds + q * SQ;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = p + P * u;
    const int base = (t / NS) * NS * R + (t % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) mine[lds_pad_index(base + r * NS)] = v[u + r * U];
  }
  __syncthreads();
  thread_map<NEXT_MODE, T, P>(tid, q, p);
  const float2* theirs = lds + q * SQ;
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = theirs[lds_pad_index(p + P * e)];
}

template <int N, int T, int LM, int SM, int TW>
__global__ void __launch_bounds__(T*(N / Blocking<N>::E))
fft_pass_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                const float2* __restrict__ twp, const PassArgs a) {
  // src and dst may be the same buffer (in-place passes): every element of a
  // tile is read before any element of it is written, and tiles are disjoint.
  constexpr int E = Blocking<N>::E;
  constexpr int P = N / E;
  constexpr int NST = num_stages<N>();
  constexpr int R0 = Blocking<N>::R0, R1 = Blocking<N>::R1, R2 = Blocking<N>::R2;
  constexpr int SQ = lds_pencil_stride<N, T>();
  constexpr int LDS_ELEMS = NST > 1 ? T * SQ : 1;
  __shared__ float2 lds[LDS_ELEMS];

  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  int q, p;
  thread_map<(NST > 1 ? LM : SM), T, P>(tid, q, p);

  float2 v[E];
  {
    const int64_t b = tile * T + q;
    if (b < a.B) {
      const float2* s =
          src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = s[(int64_t)(p + P * e) * a.ijs];
      if (a.conj_in) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e].y = -v[e].y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = make_float2(0.f, 0.f);
    }
  }

  radix_stage<N, E, P, 1, R0>(v, p, tw);
  if constexpr (NST == 2) {
    lds_exchange<N, E, P, T, SQ, 1, R0, SM>(v, lds, tid, q, p);
    radix_stage<N, E, P, R0, R1>(v, p, tw);
  } else if constexpr (NST == 3) {
    lds_exchange<N, E, P, T, SQ, 1, R0, MODE_ROW>(v, lds, tid, q, p);
    radix_stage<N, E, P, R0, R1>(v, p, tw);
    __syncthreads();  // every read of the first exchange is done
    lds_exchange<N, E, P, T, SQ, R0, R1, SM>(v, lds, tid, q, p);
    radix_stage<N, E, P, R0 * R1, R2>(v, p, tw);
  }

  const int64_t b = tile * T + q;
  if (b < a.B) {
    float2* d = dst + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    int64_t res = 0;
    if constexpr (TW) res = (b >> a.res_shift) & a.res_mask;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = p + P * e;
      float2 val = v[e];
      if constexpr (TW) val = cmul(val, twp[(res * k) & a.twp_mask]);
      if (a.conj_out) val.y = -val.y;
      d[(int64_t)k * a.oks] = val;
    }
  }
}

template <int N, int T, int LM, int SM, int TW>
hipError_t launch_pass(const PassArgs& a, const float2* src, float2* dst,
                       const float2* tw, const float2* twp, hipStream_t stream) {
  constexpr int THREADS = T * (N / Blocking<N>::E);
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_pass_kernel<N, T, LM, SM, TW>), dim3((unsigned)blocks),
                     dim3(THREADS), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int N, int T, int LM, int SM, int TW>
KernelInfo kernel_info() {
  constexpr int E = Blocking<N>::E;
  constexpr int SQ = lds_pencil_stride<N, T>();
  constexpr int LDS = num_stages<N>() > 1 ? T * SQ * 8 : 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(T * (N / E) <= 1024, "workgroup too large");
  return KernelInfo{N, T, LM, SM, TW, T * (N / E), LDS, &launch_pass<N, T, LM, SM, TW>};
}

// All four layout combinations used by the schedules for one (N, T):
//   ROW->COL  pencil pass with rotate-on-write, four-step second half;
//   ROW->ROW  contiguous axis in place (slab rows);
//   COL->COL  strided axis in place (slab columns, four-step halves);
//   COL->COL with the four-step twiddle (first half of a split axis).
template <int N, int T>
void add_kernels(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info<N, T, MODE_ROW, MODE_COL, 0>());
  v.push_back(kernel_info<N, T, MODE_ROW, MODE_ROW, 0>());
  v.push_back(kernel_info<N, T, MODE_COL, MODE_COL, 0>());
  v.push_back(kernel_info<N, T, MODE_COL, MODE_COL, 1>());
}

}  // namespace dft3d
