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

// Blocking with 64 elements per thread for the persistent 2048 kernel: a
// tile of 8 pencils runs on 256 threads (one wave per SIMD), whose register
// budget holds the current and the prefetched tile without scratch.
template <int N> struct BlockingWide;
template <> struct BlockingWide<2048> {
  static constexpr int E = 64, R0 = 64, R1 = 32, R2 = 1;
};

template <class BL> constexpr int num_stages() {
  return BL::R1 == 1 ? 1 : (BL::R2 == 1 ? 2 : 3);
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

// 8-byte global accesses, optionally marked non-temporal (streamed through
// the caches without being kept).
__device__ __forceinline__ float2 load_c64(const float2* p, bool nt) {
  if (nt) {
    const unsigned long long u =
        __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
    return __builtin_bit_cast(float2, u);
  }
  return *p;
}
__device__ __forceinline__ void store_c64(float2* p, float2 v, bool nt) {
  if (nt) {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v),
                                reinterpret_cast<unsigned long long*>(p));
  } else {
    *p = v;
  }
}

// MV (move only): the stage is left out (no twiddles, no butterflies), so a
// pass moves its data exactly as the full pass does and nothing else.
template <int N, int E, int P, int NS, int R, bool MV = false>
__device__ __forceinline__ void radix_stage(float2 (&v)[E], int p,
                                            const float2* __restrict__ tw) {
  if constexpr (MV) return;
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

// Load the tile's T pencils (thread (q, p) gets elements p + P e).  In ROW
// mode the pencil is contiguous (element stride 1 by construction).  Pencils
// past the end of a ragged last tile read the last pencil instead (always in
// bounds; their results are never stored), so the loads carry no branch.
// Inputs are conjugated (inverse transform) later, in transform_store_tile.
// Streaming (non-temporal) accesses of a pass kernel, by its NT parameter:
// 0 none, 1 loads and stores, 2 loads only, 3 stores only.  The one-sided
// forms serve passes whose other side is meant to stay in the caches.
// Bit 2 of NT (NT = 4..7) selects the move-only form of a pass kernel:
// the same loads, LDS exchanges and stores with the radix stages removed.
constexpr bool nt_loads(int nt) { return (nt & 3) == 1 || (nt & 3) == 2; }
constexpr bool nt_stores(int nt) { return (nt & 3) == 1 || (nt & 3) == 3; }
constexpr bool move_only(int nt) { return (nt & 4) != 0; }

template <int N, int T, int E, int P, int LM, int NT>
__device__ __forceinline__ void load_tile(float2 (&v)[E], const float2* src, const PassArgs& a,
                                          int64_t tile, int q, int p) {
  int64_t b = tile * T + q;
  b = b < a.B ? b : a.B - 1;
  const float2* s = src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
  const int64_t step = LM == MODE_ROW ? P : (int64_t)P * a.ijs;
  s += LM == MODE_ROW ? (int64_t)p : (int64_t)p * a.ijs;
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = load_c64(s + e * step, nt_loads(NT));
}

// Radix stages, LDS exchanges and the store of one tile whose elements are
// already in v (load mapping).  tw may point to global memory or to LDS.
template <int N, class BL, int T, int LM, int SM, int TW, int NT, int E, int P, int SQ>
__device__ __forceinline__ void transform_store_tile(float2 (&v)[E], float2* dst,
                                                     const float2* tw, const float2* twp,
                                                     float2* lds, const PassArgs& a,
                                                     int64_t tile, int tid, int q, int p) {
  constexpr int NST = num_stages<BL>();
  constexpr int R0 = BL::R0, R1 = BL::R1, R2 = BL::R2;
  constexpr bool MV = move_only(NT);
  // inverse as conj(DFT(conj(x))); applied here, where the tile is first
  // used, so that a prefetched tile is not waited for early
  if (a.conj_in) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e].y = -v[e].y;
  }
  radix_stage<N, E, P, 1, R0, MV>(v, p, tw);
  if constexpr (NST == 2) {
    lds_exchange<N, E, P, T, SQ, 1, R0, SM>(v, lds, tid, q, p);
    radix_stage<N, E, P, R0, R1, MV>(v, p, tw);
  } else if constexpr (NST == 3) {
    lds_exchange<N, E, P, T, SQ, 1, R0, MODE_ROW>(v, lds, tid, q, p);
    radix_stage<N, E, P, R0, R1, MV>(v, p, tw);
    __syncthreads();  // every read of the first exchange is done
    lds_exchange<N, E, P, T, SQ, R0, R1, SM>(v, lds, tid, q, p);
    radix_stage<N, E, P, R0 * R1, R2, MV>(v, p, tw);
  }
  const int64_t b = tile * T + q;
  if (b < a.B) {
    float2* d = dst + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    int64_t res = 0;
    if constexpr (TW) res = (b >> a.res_shift) & a.res_mask;
    const int64_t step = SM == MODE_ROW ? P : (int64_t)P * a.oks;
    d += SM == MODE_ROW ? (int64_t)p : (int64_t)p * a.oks;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = p + P * e;
      if constexpr (TW && !MV) v[e] = cmul(v[e], twp[(res * k) & a.twp_mask]);
      if (a.conj_out) v[e].y = -v[e].y;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) store_c64(d + e * step, v[e], nt_stores(NT));
  }
}

// One workgroup per tile.
template <int N, int T, int LM, int SM, int TW, int NT>
__global__ void __launch_bounds__(T*(N / Blocking<N>::E))
fft_pass_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                const float2* __restrict__ twp, const PassArgs a) {
  // src and dst may be the same buffer (in-place passes): every element of a
  // tile is read before any element of it is written, and tiles are disjoint.
  using BL = Blocking<N>;
  constexpr int E = BL::E;
  constexpr int P = N / E;
  constexpr int NST = num_stages<BL>();
  constexpr int SQ = lds_pencil_stride<N, T>();
  constexpr int LDS_ELEMS = NST > 1 ? T * SQ : 1;
  __shared__ float2 lds[LDS_ELEMS];

  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  int q, p;
  thread_map<(NST > 1 ? LM : SM), T, P>(tid, q, p);
  float2 v[E];
  load_tile<N, T, E, P, LM, NT>(v, src, a, tile, q, p);
  transform_store_tile<N, BL, T, LM, SM, TW, NT, E, P, SQ>(v, dst, tw, twp, lds, a, tile,
                                                           tid, q, p);
}

// Persistent form: a grid of about one resident workgroup per CU walks the
// tiles (virtual tile w, w + G, w + 2G, ... for workgroup w, remapped so
// that each XCD takes a contiguous range) and loads tile i+1 into registers
// while tile i goes through its stages, so the memory system never waits
// for a workgroup to finish its arithmetic.  The stage twiddles are copied
// to LDS once, keeping their reads off the vector-memory queue.
template <int N, int T, int LM, int SM, int TW, int NT, class BL>
__global__ void __launch_bounds__(T*(N / BL::E))
fft_pass_persistent(const float2* src, float2* dst, const float2* __restrict__ tw,
                    const float2* __restrict__ twp, const PassArgs a) {
  constexpr int E = BL::E;
  constexpr int P = N / E;
  constexpr int NTHR = T * P;
  constexpr int NST = num_stages<BL>();
  static_assert(NST > 1, "persistent form is for multi-stage lengths");
  constexpr int SQ = lds_pencil_stride<N, T>();
  __shared__ float2 lds[T * SQ];
  __shared__ float2 ltw[N];

  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NTHR) ltw[i] = tw[i];
  __syncthreads();

  const int64_t ntiles = (a.B + T - 1) / T;
  const int64_t G = gridDim.x;
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  int q0, p0;
  thread_map<LM, T, P>(tid, q0, p0);
  // Two register tiles in alternation (loop unrolled by two, so no copies):
  // the next tile's loads are issued before the current tile's arithmetic.
  // Past the last tile the prefetch re-reads the last tile (in bounds).
  const int64_t last = ntiles - 1;
  float2 ra[E], rb[E];
  load_tile<N, T, E, P, LM, NT>(ra, src, a, tile_index(w, ntiles, a.xcd_remap), q0, p0);
  while (true) {
    int64_t wn = w + G;
    load_tile<N, T, E, P, LM, NT>(rb, src, a, tile_index(wn < last ? wn : last, ntiles, a.xcd_remap),
                              q0, p0);
    {
      int q = q0, p = p0;
      transform_store_tile<N, BL, T, LM, SM, TW, NT, E, P, SQ>(
          ra, dst, ltw, twp, lds, a, tile_index(w, ntiles, a.xcd_remap), tid, q, p);
    }
    __syncthreads();  // LDS of this tile fully read before the next writes
    w = wn;
    if (w >= ntiles) break;
    wn = w + G;
    load_tile<N, T, E, P, LM, NT>(ra, src, a, tile_index(wn < last ? wn : last, ntiles, a.xcd_remap),
                              q0, p0);
    {
      int q = q0, p = p0;
      transform_store_tile<N, BL, T, LM, SM, TW, NT, E, P, SQ>(
          rb, dst, ltw, twp, lds, a, tile_index(w, ntiles, a.xcd_remap), tid, q, p);
    }
    __syncthreads();
    w = wn;
    if (w >= ntiles) break;
  }
}

template <int N, int T, int LM, int SM, int TW, int NT>
hipError_t launch_pass(const PassArgs& a, const float2* src, float2* dst,
                       const float2* tw, const float2* twp, hipStream_t stream) {
  constexpr int THREADS = T * (N / Blocking<N>::E);
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_pass_kernel<N, T, LM, SM, TW, NT>), dim3((unsigned)blocks),
                     dim3(THREADS), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

int device_cu_count();

template <int N, int T, int LM, int SM, int TW, int NT, class BL>
hipError_t launch_persistent(const PassArgs& a, const float2* src, float2* dst,
                             const float2* tw, const float2* twp, hipStream_t stream) {
  constexpr int THREADS = T * (N / BL::E);
  const int64_t tiles = (a.B + T - 1) / T;
  if (tiles <= 0) return hipSuccess;
  static int per_cu = -1;  // resident workgroups per CU for this kernel
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fft_pass_persistent<N, T, LM, SM, TW, NT, BL>, THREADS, 0) != hipSuccess)
      return hipGetLastError();
    per_cu = nb > 0 ? nb : 1;
  }
  int64_t grid = (int64_t)device_cu_count() * per_cu;
  if (grid > tiles) grid = tiles;
  hipLaunchKernelGGL((fft_pass_persistent<N, T, LM, SM, TW, NT, BL>), dim3((unsigned)grid),
                     dim3(THREADS), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <class BL>
void set_radices(KernelInfo& k) {
  k.r0 = BL::R0;
  k.r1 = BL::R1;
  k.r2 = BL::R2;
}

template <int N, int T, int LM, int SM, int TW, int NT, class BL>
KernelInfo kernel_info_persistent() {
  constexpr int E = BL::E;
  constexpr int SQ = lds_pencil_stride<N, T>();
  constexpr int LDS = (T * SQ + N) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  KernelInfo k{N, T, LM, SM, TW, T * (N / E), LDS,
               &launch_persistent<N, T, LM, SM, TW, NT, BL>, 1, NT & 3};
  k.move_only = move_only(NT) ? 1 : 0;
  set_radices<BL>(k);
  return k;
}

template <int N, int T, int LM, int SM, int TW, int NT>
KernelInfo kernel_info() {
  constexpr int E = Blocking<N>::E;
  constexpr int SQ = lds_pencil_stride<N, T>();
  constexpr int LDS = num_stages<Blocking<N>>() > 1 ? T * SQ * 8 : 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(T * (N / E) <= 1024, "workgroup too large");
  KernelInfo k{N, T, LM, SM, TW, T * (N / E), LDS, &launch_pass<N, T, LM, SM, TW, NT>, 0,
               NT & 3};
  k.move_only = move_only(NT) ? 1 : 0;
  set_radices<Blocking<N>>(k);
  return k;
}

// All four layout combinations used by the schedules for one (N, T):
//   ROW->COL  pencil pass with rotate-on-write, four-step second half;
//   ROW->ROW  contiguous axis in place (slab rows);
//   COL->COL  strided axis in place (slab columns, four-step halves);
//   COL->COL with the four-step twiddle (first half of a split axis).
template <int N, int T, int NT>
void add_kernels_nt(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info<N, T, MODE_ROW, MODE_COL, 0, NT>());
  v.push_back(kernel_info<N, T, MODE_ROW, MODE_ROW, 0, NT>());
  v.push_back(kernel_info<N, T, MODE_COL, MODE_COL, 0, NT>());
  v.push_back(kernel_info<N, T, MODE_COL, MODE_COL, 1, NT>());
}
// With their move-only forms (NT + 4): the same data movement without the
// radix stages, for the time breakdown of a pass.
template <int N, int T>
void add_kernels(std::vector<KernelInfo>& v) {
  add_kernels_nt<N, T, 0>(v);
  add_kernels_nt<N, T, 1>(v);
  add_kernels_nt<N, T, 4>(v);
  add_kernels_nt<N, T, 5>(v);
}

// ROW->ROW with the four-step twiddle: the first half of a split axis whose
// input is in the shuffled (digit-exchanged) order, contiguous case.
template <int N, int T>
void add_row_twiddle_kernels(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info<N, T, MODE_ROW, MODE_ROW, 1, 0>());
  v.push_back(kernel_info<N, T, MODE_ROW, MODE_ROW, 1, 1>());
}

template <int N, int T, int NT, class BL>
void add_persistent_kernels_nt(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_persistent<N, T, MODE_ROW, MODE_COL, 0, NT, BL>());
  v.push_back(kernel_info_persistent<N, T, MODE_ROW, MODE_ROW, 0, NT, BL>());
  v.push_back(kernel_info_persistent<N, T, MODE_COL, MODE_COL, 0, NT, BL>());
}
template <int N, int T, class BL = Blocking<N>>
void add_persistent_kernels(std::vector<KernelInfo>& v) {
  add_persistent_kernels_nt<N, T, 0, BL>(v);
  add_persistent_kernels_nt<N, T, 1, BL>(v);
  add_persistent_kernels_nt<N, T, 4, BL>(v);
  add_persistent_kernels_nt<N, T, 5, BL>(v);
}

// A plain copy of the B * N points of a pass from src to dst (streaming
// 16-byte accesses, two points each, or 8-byte ones for an odd point count;
// grid-stride loop): the HBM floor a pass of that size can reach, used by
// the move-only option's copy mode.
template <class V>
__global__ void __launch_bounds__(256)
copy_pass_kernel(const V* __restrict__ src, V* __restrict__ dst, int64_t count) {
  // chunks of 256 x 8 elements: each thread issues its 8 loads before its
  // stores, every load and store instruction coalesced across the wave
  constexpr int U = 8;
  const int64_t chunks = (count + 256 * U - 1) / (256 * U);
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t base = c * 256 * U + threadIdx.x;
    V x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * 256;
      if (i < count) x[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * 256;
      if (i < count) __builtin_nontemporal_store(x[u], dst + i);
    }
  }
}

template <int N>
hipError_t launch_copy(const PassArgs& a, const float2* src, float2* dst, const float2*,
                       const float2*, hipStream_t stream) {
  const int64_t count = a.B * N;
  if (count <= 0) return hipSuccess;
  const int64_t cap = (int64_t)device_cu_count() * 32;
  if (count % 2 == 0) {
    int64_t blocks = (count / 2 + 2047) / 2048;
    if (blocks > cap) blocks = cap;
    using V16 = float __attribute__((ext_vector_type(4)));
    hipLaunchKernelGGL(copy_pass_kernel<V16>, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<const V16*>(src), reinterpret_cast<V16*>(dst),
                       count / 2);
  } else {
    int64_t blocks = (count + 2047) / 2048;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(copy_pass_kernel<unsigned long long>, dim3((unsigned)blocks), dim3(256),
                       0, stream, reinterpret_cast<const unsigned long long*>(src),
                       reinterpret_cast<unsigned long long*>(dst), count);
  }
  return hipGetLastError();
}

template <int N>
KernelInfo kernel_info_copy() {
  KernelInfo k{N, 0, MODE_ROW, MODE_ROW, 0, 256, 0, &launch_copy<N>, 0, 1};
  k.move_only = 2;
  return k;
}

// Rotate-on-write passes with one streaming side: the first two passes of
// the grouped pencil schedule, whose intermediate (one group of planes)
// stays in the Infinity Cache between them.
template <int N, int T, class BL = Blocking<N>>
void add_group_kernels(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_persistent<N, T, MODE_ROW, MODE_COL, 0, 2, BL>());
  v.push_back(kernel_info_persistent<N, T, MODE_ROW, MODE_COL, 0, 3, BL>());
}

}  // namespace dft3d
