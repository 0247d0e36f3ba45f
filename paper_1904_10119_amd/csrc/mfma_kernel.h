// Split-precision leaves on the matrix cores.
//
// A length-N pass runs its radix-16 stages as dense real GEMMs on MFMA:
// for 16 vectors at a time (pencil, butterfly) the length-16 DFT
// (Section 2.1, eqs. (1)-(2)) is
//   Yr = [Fr | -Fi] [Xr; Xi],   Yi = [Fi | Fr] [Xr; Xi],
// two v_mfma_f32_16x16x32 products (M = 16 outputs, K = 32 real inputs,
// N = 16 vectors) with FP32 accumulation.  Both operands are split into
// bf16 or fp16 terms (F from FP64 at plan time, X in registers at run time)
// and the products of low combined order are accumulated, smallest first,
// which recovers FP32-level accuracy from 8- or 11-bit significands.  A
// leftover radix-2/4/8 stage and every twiddle run in FP32 on the vector
// ALUs.  The tile lives in LDS between stages (ping-pong buffers); the
// persistent form loads the next tile into registers meanwhile.
//
// Operand lane layout of the 16x16x32 MFMA (checked on gfx950): lane l
// holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i < 8, and
// receives D[4 (l / 16) + i][l % 16], i < 4.
#pragma once

#include "../../include/dft3d.h"
#include "pass_kernel.h"

namespace dft3d {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Leaf operand table (uploaded by the plan): for term t (0..2) and matrix
// c (0: [Fr | -Fi], 1: [Fi | Fr]), lane l's 8 values, as raw 16-bit
// patterns; bf16 terms unscaled, fp16 terms scaled by 2^(11 t).
constexpr int kLeafTableHalves = 3 * 2 * 64 * 8;

template <int PREC> struct LeafPolicy;
template <> struct LeafPolicy<DFT3D_PREC_BF16X1> { static constexpr int terms = 1, fp16 = 0; };
template <> struct LeafPolicy<DFT3D_PREC_FP16X1> { static constexpr int terms = 1, fp16 = 1; };
template <> struct LeafPolicy<DFT3D_PREC_BF16X6> { static constexpr int terms = 3, fp16 = 0; };
template <> struct LeafPolicy<DFT3D_PREC_BF16X9> { static constexpr int terms = 3, fp16 = 0; };
template <> struct LeafPolicy<DFT3D_PREC_FP16X3> { static constexpr int terms = 2, fp16 = 1; };

__device__ __forceinline__ f32x4_t mfma_bf16(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4_t mfma_f16(f16x8_t a, f16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// A operands of one lane: [term][matrix].
template <int PREC> struct LeafA {
  using vec = typename std::conditional<LeafPolicy<PREC>::fp16, f16x8_t, bf16x8_t>::type;
  vec a[3][2];
  __device__ __forceinline__ void load(const unsigned short* table, int lane) {
#pragma unroll
    for (int t = 0; t < LeafPolicy<PREC>::terms; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const unsigned short* s = table + ((t * 2 + c) * 64 + lane) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if constexpr (LeafPolicy<PREC>::fp16)
            a[t][c][i] = __builtin_bit_cast(_Float16, s[i]);
          else
            a[t][c][i] = __builtin_bit_cast(__bf16, s[i]);
        }
      }
  }
};

// Split 8 FP32 values into bf16 terms (x = b0 + b1 + b2 up to rounding of
// the last term); each residual is exact in FP32.
template <int TERMS>
__device__ __forceinline__ void split_bf16(const float (&x)[8], bf16x8_t (&b)[3]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float r = x[i];
#pragma unroll
    for (int t = 0; t < TERMS; ++t) {
      const __bf16 h = (__bf16)r;
      b[t][i] = h;
      r -= (float)h;
    }
  }
}

// Split into fp16 terms with term t scaled by 2^(11 t) (x already scaled so
// its largest component is in [2^14, 2^15)).
template <int TERMS>
__device__ __forceinline__ void split_f16(const float (&x)[8], f16x8_t (&b)[3]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float r = x[i];
#pragma unroll
    for (int t = 0; t < TERMS; ++t) {
      const _Float16 h = (_Float16)r;
      b[t][i] = h;
      r = (r - (float)h) * 2048.0f;
    }
  }
}

// Length-16 DFTs of 16 vectors: this lane supplies 8 real inputs (xs) of
// vector l % 16 (real parts of rows 8 (l/16) .. +7 for l/16 < 2, imaginary
// parts of rows 8 (l/16 - 2) .. +7 otherwise) and receives Yr, Yi of rows
// 4 (l/16) .. +3 of the same vector.
template <int PREC>
__device__ __forceinline__ void leaf16(const LeafA<PREC>& A, const float (&xs)[8],
                                       f32x4_t& yr, f32x4_t& yi) {
  constexpr int TERMS = LeafPolicy<PREC>::terms;
  const f32x4_t z = {0.f, 0.f, 0.f, 0.f};
  if constexpr (!LeafPolicy<PREC>::fp16) {
    bf16x8_t b[3];
    split_bf16<TERMS>(xs, b);
    f32x4_t r = z, i = z;
    if constexpr (PREC == DFT3D_PREC_BF16X9) {  // orders 4 and 3
      r = mfma_bf16(A.a[2][0], b[2], r); i = mfma_bf16(A.a[2][1], b[2], i);
      r = mfma_bf16(A.a[2][0], b[1], r); i = mfma_bf16(A.a[2][1], b[1], i);
      r = mfma_bf16(A.a[1][0], b[2], r); i = mfma_bf16(A.a[1][1], b[2], i);
    }
    if constexpr (TERMS == 3) {  // order 2, then order 1
      r = mfma_bf16(A.a[2][0], b[0], r); i = mfma_bf16(A.a[2][1], b[0], i);
      r = mfma_bf16(A.a[1][0], b[1], r); i = mfma_bf16(A.a[1][1], b[1], i);
      r = mfma_bf16(A.a[0][0], b[2], r); i = mfma_bf16(A.a[0][1], b[2], i);
      r = mfma_bf16(A.a[1][0], b[0], r); i = mfma_bf16(A.a[1][1], b[0], i);
      r = mfma_bf16(A.a[0][0], b[1], r); i = mfma_bf16(A.a[0][1], b[1], i);
    }
    r = mfma_bf16(A.a[0][0], b[0], r); i = mfma_bf16(A.a[0][1], b[0], i);
    yr = r;
    yi = i;
  } else {
    // per-vector power-of-two scale: the vector's 32 inputs sit in lanes
    // l, l ^ 16, l ^ 32, l ^ 48
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) m = fmaxf(m, fabsf(xs[k]));
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    const int e = m > 0.f ? __builtin_amdgcn_frexp_expf(m) : 0;  // m in [2^(e-1), 2^e)
    const float s = __builtin_amdgcn_ldexpf(1.0f, 15 - e);
    float xv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) xv[k] = xs[k] * s;
    f16x8_t b[3];
    split_f16<TERMS>(xv, b);
    f32x4_t r0 = z, i0 = z;
    if constexpr (TERMS == 2) {  // order-1 products, scaled by 2^11
      f32x4_t r1 = z, i1 = z;
      r1 = mfma_f16(A.a[1][0], b[0], r1); i1 = mfma_f16(A.a[1][1], b[0], i1);
      r1 = mfma_f16(A.a[0][0], b[1], r1); i1 = mfma_f16(A.a[0][1], b[1], i1);
      r0 = r1 * (1.0f / 2048.0f);
      i0 = i1 * (1.0f / 2048.0f);
    }
    r0 = mfma_f16(A.a[0][0], b[0], r0); i0 = mfma_f16(A.a[0][1], b[0], i0);
    const float inv = __builtin_amdgcn_ldexpf(1.0f, e - 15);
    yr = r0 * inv;
    yi = i0 * inv;
  }
}

// Number of radix-16 stages and the leftover VALU radix of a length.
template <int N> constexpr int mfma_stages() {
  int s = 0, n = N;
  while (n >= 16) {
    n /= 16;
    ++s;
  }
  return s;
}
template <int N> constexpr int mfma_rest() {
  int n = N;
  while (n >= 16) n /= 16;
  return n;
}
// Elements per tile: T = tile / N pencils.
template <int N> constexpr int mfma_tile_elems() { return N >= 2048 ? 4096 : 8192; }
// LDS layout of a tile: element x of pencil q at q * mfma_row + x + x / 32
// (one pad element per 32, so the stride-16 Stockham writes and the
// stride-N/16 row reads spread over the banks), with one more pad element
// per pencil so that consecutive pencils (COL-mode staging) start in
// different banks.
template <int N> constexpr int mfma_row() { return N + N / 32 + 1; }
template <int N> __device__ __forceinline__ int mfma_lds(int q, int x) {
  return q * mfma_row<N>() + x + (x >> 5);
}
template <int N> constexpr int mfma_buf_elems() {
  return (mfma_tile_elems<N>() / N) * mfma_row<N>();
}
// Workgroup size: one 16-vector group per lane group and round; two waves
// per SIMD for the 8192-element tiles.
template <int N> constexpr int mfma_threads() { return mfma_tile_elems<N>() >= 8192 ? 512 : 256; }

// Global -> registers: thread tid gets tile elements idx = tid + 256 e, as
// (pencil q, element j) in the load mode's order (ROW: j fastest, COL: q
// fastest), so a wavefront reads contiguous runs.  Pencils past the end of
// a ragged last tile re-read the last pencil (in bounds, never stored).
template <int N, int LM>
__device__ __forceinline__ void mfma_load(float2 (&v)[mfma_tile_elems<N>() / mfma_threads<N>()],
                                          const float2* src, const PassArgs& a, int64_t tile,
                                          int tid) {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int EPT = mfma_tile_elems<N>() / mfma_threads<N>();
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int idx = tid + mfma_threads<N>() * e;
    int q, j;
    if constexpr (LM == MODE_ROW) { q = idx / N; j = idx % N; }
    else { q = idx % T; j = idx / T; }
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    v[e] = src[pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2) +
               (int64_t)j * a.ijs];
  }
}

// Registers -> LDS tile (pencil q at q * mfma_row<N>()), conjugating for
// the inverse.
template <int N, int LM>
__device__ __forceinline__ void mfma_to_lds(const float2 (&v)[mfma_tile_elems<N>() / mfma_threads<N>()],
                                            float2* buf, int conj, int tid) {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int EPT = mfma_tile_elems<N>() / mfma_threads<N>();
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int idx = tid + mfma_threads<N>() * e;
    int q, j;
    if constexpr (LM == MODE_ROW) { q = idx / N; j = idx % N; }
    else { q = idx % T; j = idx / T; }
    float2 x = v[e];
    if (conj) x.y = -x.y;
    buf[mfma_lds<N>(q, j)] = x;
  }
}

// All stages of the tile held in buf[0]; returns the buffer index holding
// the result.  Radix-16 stages on the matrix cores, a leftover radix on the
// vector ALUs; Stockham order as in the register kernels.
template <int N, int PREC>
__device__ __forceinline__ int mfma_transform(float2 (*buf)[mfma_buf_elems<N>()],
                                              const float2* ltw, const LeafA<PREC>& A,
                                              int tid) {
  constexpr int TE = mfma_tile_elems<N>();
  constexpr int T = TE / N;
  constexpr int S16 = mfma_stages<N>();
  constexpr int REST = mfma_rest<N>();
  constexpr int NTHR = mfma_threads<N>();
  constexpr int ROUNDS = TE / 16 / NTHR;  // 16-vector groups: 4 per wave per round
  const int lane = tid & 63, wave = tid >> 6;
  int cur = 0;
  int NS = 1;
#pragma unroll
  for (int st = 0; st < S16; ++st) {
    const float2* in = buf[cur];
    float2* out = buf[cur ^ 1];
    const int h = lane >> 4, n = lane & 15;
    // lanes l and l + 32 feed the same eight rows of vector n (real parts
    // in lane l, imaginary parts in lane l + 32); each reads and twiddles
    // four of them and the halves are exchanged across the 32-lane boundary
    const int rb = 8 * (h & 1) + 4 * (lane >> 5);
    constexpr int stride = N / 16;  // butterflies per pencil
    const int twstep = N / (NS * 16);
#pragma unroll
    for (int ro = 0; ro < ROUNDS; ++ro) {
#pragma unroll
      for (int g4 = 0; g4 < 4; ++g4) {
        const int g = ro * NTHR + wave * 64 + g4 * 16 + n;  // vector index
        const int q = g / stride, t = g % stride;
        const int tm = t & (NS - 1);
        float xs[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int r = rb + k;
          float2 v = in[mfma_lds<N>(q, t + r * stride)];
          if (NS > 1) v = cmul(v, ltw[tm * r * twstep]);
          // lane < 32 keeps its real part and gets the partner's; lane >= 32
          // gets the partner's imaginary part and keeps its own
          const auto sw = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, v.x),
                                                           __builtin_bit_cast(unsigned, v.y),
                                                           false, false);
          xs[k] = __builtin_bit_cast(float, (unsigned)sw[0]);
          xs[4 + k] = __builtin_bit_cast(float, (unsigned)sw[1]);
        }
        f32x4_t yr, yi;
        leaf16<PREC>(A, xs, yr, yi);
        const int base = (t / NS) * NS * 16 + tm;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rp = 4 * h + i;
          out[mfma_lds<N>(q, base + rp * NS)] = make_float2(yr[i], yi[i]);
        }
      }
    }
    __syncthreads();
    cur ^= 1;
    NS *= 16;
  }
  if constexpr (REST > 1) {  // last stage on the vector ALUs
    const float2* in = buf[cur];
    float2* out = buf[cur ^ 1];
    constexpr int BF = N / REST;  // butterflies per pencil
    const int twstep = N / (NS * REST);
    for (int idx = tid; idx < T * BF; idx += NTHR) {
      const int q = idx / BF, t = idx % BF;
      const int tm = t & (NS - 1);
      float2 v[REST];
#pragma unroll
      for (int r = 0; r < REST; ++r) {
        v[r] = in[mfma_lds<N>(q, t + r * BF)];
        if (r > 0 && NS > 1) v[r] = cmul(v[r], ltw[tm * r * twstep]);
      }
      dft<REST>(v);
      const int base = (t / NS) * NS * REST + tm;
#pragma unroll
      for (int r = 0; r < REST; ++r) out[mfma_lds<N>(q, base + r * NS)] = v[r];
    }
    __syncthreads();
    cur ^= 1;
  }
  return cur;
}

// LDS result -> global, in the store mode's order.
template <int N, int SM>
__device__ __forceinline__ void mfma_store(const float2* res, float2* dst, const PassArgs& a,
                                           int64_t tile, int tid) {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int EPT = mfma_tile_elems<N>() / mfma_threads<N>();
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int idx = tid + mfma_threads<N>() * e;
    int q, k;
    if constexpr (SM == MODE_ROW) { q = idx / N; k = idx % N; }
    else { q = idx % T; k = idx / T; }
    const int64_t b = tile * T + q;
    float2 v = res[mfma_lds<N>(q, k)];
    if (a.conj_out) v.y = -v.y;
    if (b < a.B)
      dst[pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2) + (int64_t)k * a.oks] =
          v;
  }
}

// One tile per workgroup: all loads of the tile are issued before any is
// written to LDS, so a workgroup keeps 32 loads per thread in flight.
template <int N, int LM, int SM, int PREC>
__global__ void __launch_bounds__(mfma_threads<N>())
fft_pass_mfma(const float2* src, float2* dst, const float2* __restrict__ tw,
              const unsigned short* __restrict__ leaf, const PassArgs a) {
  constexpr int EPT = mfma_tile_elems<N>() / mfma_threads<N>();
  __shared__ float2 buf[2][mfma_buf_elems<N>()];
  __shared__ float2 ltw[N];
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  float2 v[EPT];
  mfma_load<N, LM>(v, src, a, tile, tid);
  for (int i = tid; i < N; i += mfma_threads<N>()) ltw[i] = tw[i];
  LeafA<PREC> A;
  A.load(leaf, tid & 63);
  mfma_to_lds<N, LM>(v, buf[0], a.conj_in, tid);
  __syncthreads();
  const int cur = mfma_transform<N, PREC>(buf, ltw, A, tid);
  mfma_store<N, SM>(buf[cur], dst, a, tile, tid);
}

// Persistent form: about one resident workgroup per CU walks the tiles
// (w, w + G, ...; remapped per XCD).  The next tile's loads go out as soon
// as the current tile is in LDS, so they are in flight during its matrix-
// core stages and its stores.
template <int N, int LM, int SM, int PREC>
__global__ void __launch_bounds__(mfma_threads<N>())
fft_pass_mfma_persistent(const float2* src, float2* dst, const float2* __restrict__ tw,
                         const unsigned short* __restrict__ leaf, const PassArgs a) {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int EPT = mfma_tile_elems<N>() / mfma_threads<N>();
  __shared__ float2 buf[2][mfma_buf_elems<N>()];
  __shared__ float2 ltw[N];
  const int tid = threadIdx.x;
  const int64_t ntiles = (a.B + T - 1) / T;
  const int64_t G = gridDim.x;
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  const int64_t last = ntiles - 1;
  float2 v[EPT];
  mfma_load<N, LM>(v, src, a, tile_index(w, ntiles, a.xcd_remap), tid);
  for (int i = tid; i < N; i += mfma_threads<N>()) ltw[i] = tw[i];
  LeafA<PREC> A;
  A.load(leaf, tid & 63);
  while (true) {
    mfma_to_lds<N, LM>(v, buf[0], a.conj_in, tid);
    __syncthreads();
    const int64_t wn = w + G;
    // prefetch the next tile (past the end: the last tile again, in bounds)
    mfma_load<N, LM>(v, src, a, tile_index(wn < last ? wn : last, ntiles, a.xcd_remap), tid);
    const int cur = mfma_transform<N, PREC>(buf, ltw, A, tid);
    mfma_store<N, SM>(buf[cur], dst, a, tile_index(w, ntiles, a.xcd_remap), tid);
    __syncthreads();  // every read of the result buffer is done
    w = wn;
    if (w >= ntiles) break;
  }
}

template <int N, int LM, int SM, int PREC>
hipError_t launch_mfma(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                       const float2* leaf, hipStream_t stream) {
  constexpr int T = mfma_tile_elems<N>() / N;
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_pass_mfma<N, LM, SM, PREC>), dim3((unsigned)blocks),
                     dim3(mfma_threads<N>()), 0, stream, src, dst, tw,
                     reinterpret_cast<const unsigned short*>(leaf), a);
  return hipGetLastError();
}

template <int N, int LM, int SM, int PREC>
hipError_t launch_mfma_persistent(const PassArgs& a, const float2* src, float2* dst,
                                  const float2* tw, const float2* leaf, hipStream_t stream) {
  constexpr int T = mfma_tile_elems<N>() / N;
  const int64_t tiles = (a.B + T - 1) / T;
  if (tiles <= 0) return hipSuccess;
  static int per_cu = -1;  // resident workgroups per CU for this kernel
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fft_pass_mfma_persistent<N, LM, SM, PREC>, mfma_threads<N>(), 0) != hipSuccess)
      return hipGetLastError();
    per_cu = nb > 0 ? nb : 1;
  }
  int64_t grid = (int64_t)device_cu_count() * per_cu;
  if (grid > tiles) grid = tiles;
  hipLaunchKernelGGL((fft_pass_mfma_persistent<N, LM, SM, PREC>), dim3((unsigned)grid),
                     dim3(mfma_threads<N>()), 0, stream, src, dst, tw,
                     reinterpret_cast<const unsigned short*>(leaf), a);
  return hipGetLastError();
}

template <int N, int LM, int SM, int PREC, int PERS>
KernelInfo kernel_info_mfma() {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int LDS = (2 * mfma_buf_elems<N>() + N) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(mfma_tile_elems<N>() % (16 * mfma_threads<N>()) == 0, "whole rounds");
  return KernelInfo{N, T, LM, SM, 0, mfma_threads<N>(), LDS,
                    PERS ? &launch_mfma_persistent<N, LM, SM, PREC> : &launch_mfma<N, LM, SM, PREC>,
                    PERS, 0, PREC};
}

template <int N, int PREC>
void add_mfma_kernels_prec(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_COL, PREC, 0>());
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_ROW, PREC, 0>());
  v.push_back(kernel_info_mfma<N, MODE_COL, MODE_COL, PREC, 0>());
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_COL, PREC, 1>());
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_ROW, PREC, 1>());
  v.push_back(kernel_info_mfma<N, MODE_COL, MODE_COL, PREC, 1>());
}

template <int N>
void add_mfma_kernels(std::vector<KernelInfo>& v) {
  add_mfma_kernels_prec<N, DFT3D_PREC_BF16X1>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_FP16X1>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_BF16X6>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_BF16X9>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_FP16X3>(v);
}

}  // namespace dft3d
