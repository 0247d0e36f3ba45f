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
// ALUs.  The first stage takes its operands straight from the registers
// the tile was loaded into, later stages run in LDS (in place in the
// one-tile form, ping-pong between two buffers in the persistent form), and
// a leftover radix writes straight to global memory; the persistent form
// loads the next tile into registers meanwhile.
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
// sgn (+1 or -1) is the vector's sign (see mfma_vector_sign), folded into
// the power-of-two scale and its inverse: both exact.
template <int PREC>
__device__ __forceinline__ void leaf16(const LeafA<PREC>& A, const float (&xs)[8], float sgn,
                                       f32x4_t& yr, f32x4_t& yi) {
  constexpr int TERMS = LeafPolicy<PREC>::terms;
  const f32x4_t z = {0.f, 0.f, 0.f, 0.f};
  // Per-vector power-of-two scale (exact): the vector's 32 inputs sit in
  // lanes l, l ^ 16, l ^ 32, l ^ 48; its largest component is brought to
  // [2^14, 2^15).  fp16 terms need it for the format's range; bf16 terms
  // share FP32's exponent range but need it for tiny vectors (below about
  // 2^-100), whose residuals would otherwise fall into the subnormal range
  // and lose bits or be flushed by the matrix cores.  The maximum over the
  // four lanes comes from two lane swaps (v_permlane32_swap: lanes l and
  // l ^ 32; v_permlane16_swap: rows 2j and 2j + 1, i.e. l and l ^ 16), no
  // LDS round trip.  e is kept at -100 or above so that the scale
  // 2^(15 - e) stays finite (a vector below 2^-101 is scaled by 2^115:
  // smaller than ideal, never inf or NaN).
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) m = fmaxf(m, fabsf(xs[k]));
  {
    const unsigned u = __builtin_bit_cast(unsigned, m);
    const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    m = fmaxf(__builtin_bit_cast(float, (unsigned)h[0]), __builtin_bit_cast(float, (unsigned)h[1]));
    const unsigned w = __builtin_bit_cast(unsigned, m);
    const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
    m = fmaxf(__builtin_bit_cast(float, (unsigned)r[0]), __builtin_bit_cast(float, (unsigned)r[1]));
  }
  int e = m > 0.f ? __builtin_amdgcn_frexp_expf(m) : 0;  // m in [2^(e-1), 2^e)
  e = e < -100 ? -100 : e;
  const float sc = __builtin_amdgcn_ldexpf(sgn, 15 - e);
  const float inv = __builtin_amdgcn_ldexpf(sgn, e - 15);
  float xv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) xv[k] = xs[k] * sc;
  if constexpr (!LeafPolicy<PREC>::fp16) {
    bf16x8_t b[3];
    split_bf16<TERMS>(xv, b);
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
    yr = r * inv;
    yi = i * inv;
  } else {
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
template <int N> constexpr int mfma_tile_elems() { return N >= 4096 ? 4096 : 8192; }
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
// Workgroup size: one 16-vector group per lane group, so one round of
// 16-vector groups covers the tile (two waves per SIMD for 8192 points).
template <int N> constexpr int mfma_threads() { return mfma_tile_elems<N>() / 16; }
// Tile elements each lane holds for the first stage (4 groups x 4 rows).
constexpr int kMfmaRegs = 16;

// Vector (pencil q, butterfly t) of a 16-vector group index g.  For the
// first stage the load mode's contiguous index runs fastest across lanes
// (ROW: t, COL: q), so the operands come straight from global memory in
// 128-byte runs; later stages use the ROW order.
template <int N, int MODE>
__device__ __forceinline__ void mfma_vec(int g, int& q, int& t) {
  constexpr int stride = N / 16;
  constexpr int T = mfma_tile_elems<N>() / N;
  if constexpr (MODE == MODE_ROW) { q = g / stride; t = g % stride; }
  else { q = g % T; t = g / T; }
}

// Global -> registers, already in first-stage operand order: lane (wave,
// n, h, half) gets rows rb .. rb + 3 (rb = 8 (h & 1) + 4 half) of vector
// g = wave * 64 + g4 * 16 + n for g4 < 4.  Pencils past the end of a ragged
// last tile re-read the last pencil (in bounds, never stored).
template <int N, int LM>
__device__ __forceinline__ void mfma_load(float2 (&v)[kMfmaRegs], const float2* src,
                                          const PassArgs& a, int64_t tile, int tid) {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int stride = N / 16;
  const int lane = tid & 63, wave = tid >> 6;
  const int rb = 8 * ((lane >> 4) & 1) + 4 * (lane >> 5);
  // element stride along the pencil: 1 in ROW mode (by construction)
  const int64_t js = LM == MODE_ROW ? 1 : a.ijs;
#pragma unroll
  for (int g4 = 0; g4 < 4; ++g4) {
    int q, t;
    mfma_vec<N, LM>(wave * 64 + g4 * 16 + (lane & 15), q, t);
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    const float2* s = src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2) +
                      (int64_t)(t + rb * stride) * js;
    const int64_t step = (int64_t)stride * js;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[g4 * 4 + k] = s[k * step];
  }
}

// One radix-16 stage for the lane's four 16-vector groups.  x[g4 * 4 + k]
// is row rb + k of group g4's vector, already twiddled; lanes l and l + 32
// hold the same vector's rows 0..3 and 4..7 (of the lane group's eight) and
// exchange halves across the 32-lane boundary so that lane l feeds real
// parts and lane l + 32 imaginary parts to the matrix cores.
//
// The matrix cores do not round their dot products to nearest: measured on
// random operands the result carries a bias of a fraction of an ulp of one
// sign.  Summed coherently by the later stages and axes, that bias grows
// with the transform size wherever the weights of a sum line up with it: at
// the DC bins when every vector is transformed alike, and still at some
// output of a 1024^3 transform (4.6e-5 of the output rms, 2.8 times the
// per-element bar of 10 tol(N)) when every other vector by the parity of
// pencil + butterfly was transformed negated, a pattern that repeats with
// every tile.  Each vector (pencil b, butterfly t, stage NS) is therefore
// transformed with a pseudo-random sign from a hash of (b, t, NS) and the
// result multiplied by the same sign (exact operations): the biases then
// add like independent rounding errors at every output.
__device__ __forceinline__ float mfma_vector_sign(int64_t b, int t, int NS) {
  unsigned int x = (unsigned int)b * 0x9e3779b9u + (unsigned int)(t * 16 + __builtin_ctz(NS)) *
                                                       0x85ebca77u;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return (x & 0x80000000u) ? -1.0f : 1.0f;
}

template <int N, int PREC>
__device__ __forceinline__ void mfma_leaf_store(const float2 (&x)[4], const LeafA<PREC>& A,
                                                float2* out, int64_t pbase, int q, int t,
                                                int NS, int lane) {
  const float sgn = mfma_vector_sign(pbase + q, t, NS);
  float xs[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // lane < 32 keeps its real part and gets the partner's; lane >= 32
    // gets the partner's imaginary part and keeps its own
    const auto sw = __builtin_amdgcn_permlane32_swap(
        __builtin_bit_cast(unsigned, x[k].x), __builtin_bit_cast(unsigned, x[k].y), false, false);
    xs[k] = __builtin_bit_cast(float, (unsigned)sw[0]);
    xs[4 + k] = __builtin_bit_cast(float, (unsigned)sw[1]);
  }
  // the four lanes of a vector (l, l ^ 16, l ^ 32, l ^ 48) share (q, t), so
  // the sign needs no exchange
  f32x4_t yr, yi;
  leaf16<PREC>(A, xs, sgn, yr, yi);
  const int h = lane >> 4;
  const int tm = t & (NS - 1);
  const int base = (t / NS) * NS * 16 + tm;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    out[mfma_lds<N>(q, base + (4 * h + i) * NS)] = make_float2(yr[i], yi[i]);
}

// First stage from the registers mfma_load filled (conjugated for the
// inverse), output to LDS buffer out.
template <int N, int LM, int PREC>
__device__ __forceinline__ void mfma_first_stage(const float2 (&v)[kMfmaRegs], float2* out,
                                                 const LeafA<PREC>& A, int conj,
                                                 int64_t pbase, int tid) {
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int g4 = 0; g4 < 4; ++g4) {
    int q, t;
    mfma_vec<N, LM>(wave * 64 + g4 * 16 + (lane & 15), q, t);
    float2 x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = v[g4 * 4 + k];
      if (conj) x[k].y = -x[k].y;
    }
    mfma_leaf_store<N, PREC>(x, A, out, pbase, q, t, 1, lane);
  }
}

// The one-tile form's later radix-16 stages, in place in the LDS tile:
// every lane reads the inputs of its four 16-vector groups (twiddled) into
// registers, the workgroup waits, and the leaves write their outputs back to
// their Stockham places.  One buffer (not two) leaves room for two
// workgroups per CU.
template <int N, int PREC>
__device__ __forceinline__ void mfma_later_stages(float2* io, const float2* ltw,
                                                  const LeafA<PREC>& A, int64_t pbase,
                                                  int tid) {
  constexpr int S16 = mfma_stages<N>();
  constexpr int stride = N / 16;
  const int lane = tid & 63, wave = tid >> 6;
  const int rb = 8 * ((lane >> 4) & 1) + 4 * (lane >> 5);
  int NS = 16;
#pragma unroll
  for (int st = 1; st < S16; ++st) {
    const int twstep = N / (NS * 16);
    float2 x[4][4];
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      int q, t;
      mfma_vec<N, MODE_ROW>(wave * 64 + g4 * 16 + (lane & 15), q, t);
      const int tm = t & (NS - 1);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = rb + k;
        x[g4][k] = cmul(io[mfma_lds<N>(q, t + r * stride)], ltw[tm * r * twstep]);
      }
    }
    __syncthreads();  // every input of the stage is read
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      int q, t;
      mfma_vec<N, MODE_ROW>(wave * 64 + g4 * 16 + (lane & 15), q, t);
      mfma_leaf_store<N, PREC>(x[g4], A, io, pbase, q, t, NS, lane);
    }
    __syncthreads();  // every output of the stage is written
    NS *= 16;
  }
}

// The persistent form's later stages: ping-pong between two LDS buffers
// (starting from buffer 0; no wait between a stage's reads and its writes,
// and fewer registers held across the waits than in place); returns the
// buffer index holding the result.
template <int N, int PREC>
__device__ __forceinline__ int mfma_later_stages_pingpong(float2 (*buf)[mfma_buf_elems<N>()],
                                                 const float2* ltw, const LeafA<PREC>& A,
                                                 int64_t pbase, int tid) {
  constexpr int S16 = mfma_stages<N>();
  constexpr int stride = N / 16;
  const int lane = tid & 63, wave = tid >> 6;
  const int rb = 8 * ((lane >> 4) & 1) + 4 * (lane >> 5);
  int cur = 0;
  int NS = 16;
#pragma unroll
  for (int st = 1; st < S16; ++st) {
    const float2* in = buf[cur];
    float2* out = buf[cur ^ 1];
    const int twstep = N / (NS * 16);
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      int q, t;
      mfma_vec<N, MODE_ROW>(wave * 64 + g4 * 16 + (lane & 15), q, t);
      const int tm = t & (NS - 1);
      float2 x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = rb + k;
        x[k] = cmul(in[mfma_lds<N>(q, t + r * stride)], ltw[tm * r * twstep]);
      }
      mfma_leaf_store<N, PREC>(x, A, out, pbase, q, t, NS, lane);
    }
    __syncthreads();
    cur ^= 1;
    NS *= 16;
  }
  return cur;
}

// Last step: with a leftover radix, its butterflies read LDS and write
// straight to global memory (lanes ordered by the store mode's contiguous
// index); otherwise the result is copied out in the store mode's order.
template <int N, int SM>
__device__ __forceinline__ void mfma_finish(const float2* res, float2* dst, const float2* ltw,
                                            const PassArgs& a, int64_t tile, int tid) {
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int NTHR = mfma_threads<N>();
  constexpr int REST = mfma_rest<N>();
  if constexpr (REST > 1) {
    constexpr int BF = N / REST;  // butterflies per pencil == stride of the outputs
    static_assert((T * BF) % NTHR == 0, "whole butterflies per thread");
#pragma unroll
    for (int c = 0; c < T * BF / NTHR; ++c) {
      const int idx = tid + NTHR * c;
      int q, t;
      if constexpr (SM == MODE_ROW) { q = idx / BF; t = idx % BF; }
      else { q = idx % T; t = idx / T; }
      float2 v[REST];
#pragma unroll
      for (int r = 0; r < REST; ++r) {
        v[r] = res[mfma_lds<N>(q, t + r * BF)];
        if (r > 0) v[r] = cmul(v[r], ltw[t * r]);
      }
      dft<REST>(v);
      const int64_t b = tile * T + q;
      if (b < a.B) {
        // element stride along the pencil: 1 in ROW mode (by construction)
        const int64_t ks = SM == MODE_ROW ? 1 : a.oks;
        float2* d = dst + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2) +
                    (int64_t)t * ks;
        const int64_t step = (int64_t)BF * ks;
#pragma unroll
        for (int r = 0; r < REST; ++r) {
          float2 o = v[r];
          if (a.conj_out) o.y = -o.y;
          d[r * step] = o;
        }
      }
    }
  } else {
    constexpr int EPT = mfma_tile_elems<N>() / NTHR;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + NTHR * e;
      int q, k;
      if constexpr (SM == MODE_ROW) { q = idx / N; k = idx % N; }
      else { q = idx % T; k = idx / T; }
      const int64_t b = tile * T + q;
      float2 v = res[mfma_lds<N>(q, k)];
      if (a.conj_out) v.y = -v.y;
      const int64_t ks = SM == MODE_ROW ? 1 : a.oks;
      if (b < a.B)
        dst[pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2) + (int64_t)k * ks] = v;
    }
  }
}

// One tile per workgroup.
template <int N, int LM, int SM, int PREC>
__global__ void __launch_bounds__(mfma_threads<N>())
fft_pass_mfma(const float2* src, float2* dst, const float2* __restrict__ tw,
              const unsigned short* __restrict__ leaf, const PassArgs a) {
  __shared__ float2 buf[mfma_buf_elems<N>()];
  __shared__ float2 ltw[N];
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  float2 v[kMfmaRegs];
  mfma_load<N, LM>(v, src, a, tile, tid);
  for (int i = tid; i < N; i += mfma_threads<N>()) ltw[i] = tw[i];
  LeafA<PREC> A;
  A.load(leaf, tid & 63);
  constexpr int T = mfma_tile_elems<N>() / N;
  mfma_first_stage<N, LM, PREC>(v, buf, A, a.conj_in, tile * T, tid);
  __syncthreads();
  mfma_later_stages<N, PREC>(buf, ltw, A, tile * T, tid);
  mfma_finish<N, SM>(buf, dst, ltw, a, tile, tid);
}

// Persistent form: about one resident workgroup per CU walks the tiles
// (w, w + G, ...; remapped per XCD).  As soon as the first stage has
// consumed the registers, the next tile's loads go out, so they are in
// flight during the remaining stages and the stores.
template <int N, int LM, int SM, int PREC>
__global__ void __launch_bounds__(mfma_threads<N>())
fft_pass_mfma_persistent(const float2* src, float2* dst, const float2* __restrict__ tw,
                         const unsigned short* __restrict__ leaf, const PassArgs a) {
  constexpr int T = mfma_tile_elems<N>() / N;
  __shared__ float2 buf[2][mfma_buf_elems<N>()];
  __shared__ float2 ltw[N];
  const int tid = threadIdx.x;
  const int64_t ntiles = (a.B + T - 1) / T;
  const int64_t G = gridDim.x;
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  const int64_t last = ntiles - 1;
  float2 v[kMfmaRegs];
  mfma_load<N, LM>(v, src, a, tile_index(w, ntiles, a.xcd_remap), tid);
  for (int i = tid; i < N; i += mfma_threads<N>()) ltw[i] = tw[i];
  LeafA<PREC> A;
  A.load(leaf, tid & 63);
  __syncthreads();  // twiddles in LDS
  while (true) {
    const int64_t tile = tile_index(w, ntiles, a.xcd_remap);
    mfma_first_stage<N, LM, PREC>(v, buf[0], A, a.conj_in, tile * T, tid);
    __syncthreads();
    const int64_t wn = w + G;
    // prefetch the next tile (past the end: the last tile again, in bounds)
    mfma_load<N, LM>(v, src, a, tile_index(wn < last ? wn : last, ntiles, a.xcd_remap), tid);
    const int cur = mfma_later_stages_pingpong<N, PREC>(buf, ltw, A, tile * T, tid);
    mfma_finish<N, SM>(buf[cur], dst, ltw, a, tile, tid);
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
  constexpr int LDS = ((PERS ? 2 : 1) * mfma_buf_elems<N>() + N) * 8;
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
