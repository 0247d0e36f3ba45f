// Split-precision leaves on the matrix cores.
//
// A length-N pass runs its radix-16 or radix-32 stages as dense real GEMMs
// on MFMA (Section 2.1, eqs. (1)-(2)).  For 16 vectors at a time (pencil,
// butterfly) the length-16 DFT is
//   Yr = [Fr | -Fi] [Xr; Xi],   Yi = [Fi | Fr] [Xr; Xi],
// two v_mfma_f32_16x16x32 products (M = 16 outputs, K = 32 real inputs,
// N = 16 vectors) with FP32 accumulation.  The length-32 DFT of 16 vectors
// takes its even inputs xe (x[2k]) and odd inputs xo (x[2k + 1]) through
// two such products, F xe and H xo with H[p][k] = w_32^{p (2k + 1)} (the
// odd half's twiddles folded into its table), and joins them:
//   y[p] = (F xe)[p] + (H xo)[p],   y[p + 16] = (F xe)[p] - (H xo)[p].
// Both operands are split into bf16 or fp16 terms (tables from FP64 at
// plan time, X in registers at run time) and the products of low combined
// order are accumulated, smallest first, which recovers FP32-level
// accuracy from 8- or 11-bit significands.  A leftover radix-2/4/8 stage
// and every twiddle between stages run in FP32 on the vector ALUs.  The
// first stage takes its operands straight from the registers the tile was
// loaded into, later stages run in LDS (in place in the one-tile form,
// ping-pong between two buffers in the persistent form), and a leftover
// radix writes straight to global memory; the persistent form loads the
// next tile into registers meanwhile.
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

// Leaf operand table (uploaded by the plan), as raw 16-bit patterns, bf16
// terms unscaled, fp16 terms scaled by 2^(11 t): for term t (0..2) and
// matrix c (0: [Fr | -Fi], 1: [Fi | Fr]) lane l's 8 values, F[p][k] =
// w_16^{p k}; then the same for the odd-half table H[p][k] =
// w_32^{p (2k + 1)} of the length-32 leaf.
constexpr int kLeaf16Halves = 3 * 2 * 64 * 8;
constexpr int kLeafTableHalves = 2 * kLeaf16Halves;

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

// A operands of one lane for leaf length L: [term][matrix], matrices 0, 1
// of F and, for L = 32, matrices 2, 3 of H.
template <int PREC, int L = 16> struct LeafA {
  using vec = typename std::conditional<LeafPolicy<PREC>::fp16, f16x8_t, bf16x8_t>::type;
  static constexpr int C = L == 32 ? 4 : 2;
  vec a[3][C];
  __device__ __forceinline__ void load(const unsigned short* table, int lane) {
#pragma unroll
    for (int t = 0; t < LeafPolicy<PREC>::terms; ++t)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const unsigned short* s =
            table + (c >= 2 ? kLeaf16Halves : 0) + ((t * 2 + c % 2) * 64 + lane) * 8;
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

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Split 8 FP32 values into bf16 terms (x = b0 + b1 + b2 up to rounding of
// the last term); each residual is exact in FP32.  Pairs are rounded to
// nearest together (v_cvt_pk_bf16_f32) and widened back by shifts.
template <int TERMS>
__device__ __forceinline__ void split_terms(const float (&x)[8], bf16x8_t (&b)[3]) {
  u32x4_t w[3];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    float r0 = x[2 * p], r1 = x[2 * p + 1];
#pragma unroll
    for (int t = 0; t < TERMS; ++t) {
      const f32x2_t v = {r0, r1};
      const unsigned pk = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
      w[t][p] = pk;
      if (t + 1 < TERMS) {
        r0 -= __builtin_bit_cast(float, pk << 16);
        r1 -= __builtin_bit_cast(float, pk & 0xffff0000u);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TERMS; ++t) b[t] = __builtin_bit_cast(bf16x8_t, w[t]);
}

// Split into fp16 terms with term t scaled by 2^(11 t) (x already scaled so
// its largest component is in [2^14, 2^15)); pairs rounded together.
template <int TERMS>
__device__ __forceinline__ void split_terms(const float (&x)[8], f16x8_t (&b)[3]) {
  u32x4_t w[3];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    float r0 = x[2 * p], r1 = x[2 * p + 1];
#pragma unroll
    for (int t = 0; t < TERMS; ++t) {
      const f32x2_t v = {r0, r1};
      const f16x2_t h = __builtin_convertvector(v, f16x2_t);
      w[t][p] = __builtin_bit_cast(unsigned, h);
      if (t + 1 < TERMS) {
        const f32x2_t back = __builtin_convertvector(h, f32x2_t);
        r0 = (r0 - back[0]) * 2048.0f;
        r1 = (r1 - back[1]) * 2048.0f;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TERMS; ++t) b[t] = __builtin_bit_cast(f16x8_t, w[t]);
}

__device__ __forceinline__ f32x4_t mfma_op(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return mfma_bf16(a, b, c);
}
__device__ __forceinline__ f32x4_t mfma_op(f16x8_t a, f16x8_t b, f32x4_t c) {
  return mfma_f16(a, b, c);
}

// Per-vector power-of-two scale (exact), with the vector's sign sgn (+1 or
// -1, see mfma_vector_sign) folded into it and its inverse: the vector's
// inputs sit in lanes l, l ^ 16, l ^ 32, l ^ 48; its largest component is
// brought to [2^14, 2^15).  fp16 terms need it for the format's range;
// bf16 terms share FP32's exponent range but need it for tiny vectors
// (below about 2^-100), whose residuals would otherwise fall into the
// subnormal range and lose bits or be flushed by the matrix cores.  The
// maximum over the four lanes comes from two lane swaps
// (v_permlane32_swap: lanes l and l ^ 32; v_permlane16_swap: rows 2j and
// 2j + 1, i.e. l and l ^ 16), no LDS round trip.  e is kept at -100 or
// above so that the scale 2^(15 - e) stays finite (a vector below 2^-101 is
// scaled by 2^115: smaller than ideal, never inf or NaN).
template <int NV>
__device__ __forceinline__ void vector_scale(const float (&xs)[NV], float sgn, float& sc,
                                             float& inv) {
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < NV; ++k) m = fmaxf(m, fabsf(xs[k]));
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
  sc = __builtin_amdgcn_ldexpf(sgn, 15 - e);
  inv = __builtin_amdgcn_ldexpf(sgn, e - 15);
}

// The split products of K accumulators, smallest combined order first:
// prod(ta, tb, acc) accumulates table term ta times input term tb into
// every accumulator.  bf16x6 takes the six products of combined order <= 2,
// bf16x9 all nine, fp16x3 the three of order <= 1 (order 1 scaled by 2^11
// and summed on its own first).
template <int PREC, int K, class Prod>
__device__ __forceinline__ void split_products(Prod&& prod, f32x4_t (&acc)[K]) {
  constexpr int TERMS = LeafPolicy<PREC>::terms;
  const f32x4_t z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = z;
  if constexpr (!LeafPolicy<PREC>::fp16) {
    if constexpr (PREC == DFT3D_PREC_BF16X9) {  // orders 4 and 3
      prod(2, 2, acc);
      prod(2, 1, acc);
      prod(1, 2, acc);
    }
    if constexpr (TERMS == 3) {  // order 2, then order 1
      prod(2, 0, acc);
      prod(1, 1, acc);
      prod(0, 2, acc);
      prod(1, 0, acc);
      prod(0, 1, acc);
    }
  } else if constexpr (TERMS == 2) {
    f32x4_t a1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) a1[j] = z;
    prod(1, 0, a1);
    prod(0, 1, a1);
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = a1[j] * (1.0f / 2048.0f);
  }
  prod(0, 0, acc);
}

// Length-16 DFTs of 16 vectors: this lane supplies 8 real inputs (xs) of
// vector l % 16 (real parts of rows 8 (l/16) .. +7 for l/16 < 2, imaginary
// parts of rows 8 (l/16 - 2) .. +7 otherwise) and receives Yr, Yi of rows
// 4 (l/16) .. +3 of the same vector.
template <int PREC>
__device__ __forceinline__ void leaf16(const LeafA<PREC, 16>& A, const float (&xs)[8], float sgn,
                                       f32x4_t& yr, f32x4_t& yi) {
  constexpr int TERMS = LeafPolicy<PREC>::terms;
  float sc, inv;
  vector_scale(xs, sgn, sc, inv);
  float xv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) xv[k] = xs[k] * sc;
  typename LeafA<PREC, 16>::vec b[3];
  split_terms<TERMS>(xv, b);
  f32x4_t acc[2];
  split_products<PREC>(
      [&](int ta, int tb, f32x4_t(&a)[2]) {
        a[0] = mfma_op(A.a[ta][0], b[tb], a[0]);
        a[1] = mfma_op(A.a[ta][1], b[tb], a[1]);
      },
      acc);
  yr = acc[0] * inv;
  yi = acc[1] * inv;
}

// Length-32 DFTs of 16 vectors: xs[j] is row 16 (l/16 & 1) + j of the
// input (real part for l/16 < 2, imaginary part otherwise), so xs[2i] is
// row 8 (l/16 & 1) + i of xe and xs[2i + 1] the same row of xo; the lane
// receives Yr, Yi of rows 16 m + 4 (l/16) .. +3 in yr[m], yi[m].
template <int PREC>
__device__ __forceinline__ void leaf32(const LeafA<PREC, 32>& A, const float (&xs)[16],
                                       float sgn, f32x4_t (&yr)[2], f32x4_t (&yi)[2]) {
  constexpr int TERMS = LeafPolicy<PREC>::terms;
  float sc, inv;
  vector_scale(xs, sgn, sc, inv);
  float xe[8], xo[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    xe[k] = xs[2 * k] * sc;
    xo[k] = xs[2 * k + 1] * sc;
  }
  typename LeafA<PREC, 32>::vec be[3], bo[3];
  split_terms<TERMS>(xe, be);
  split_terms<TERMS>(xo, bo);
  // F xe and H xo interleaved: four independent accumulator chains
  f32x4_t acc[4];
  split_products<PREC>(
      [&](int ta, int tb, f32x4_t(&a)[4]) {
        a[0] = mfma_op(A.a[ta][0], be[tb], a[0]);
        a[1] = mfma_op(A.a[ta][1], be[tb], a[1]);
        a[2] = mfma_op(A.a[ta][2], bo[tb], a[2]);
        a[3] = mfma_op(A.a[ta][3], bo[tb], a[3]);
      },
      acc);
  const f32x4_t pr = acc[0] * inv, pi = acc[1] * inv;
  yr[0] = pr + acc[2] * inv;
  yi[0] = pi + acc[3] * inv;
  yr[1] = pr - acc[2] * inv;
  yi[1] = pi - acc[3] * inv;
}

// Stages of a length-N pass with leaf length L: every MFMA stage has radix
// L; the leftover VALU radix is below 16 (with L = 32 only lengths 32^s r,
// r < 16, are compiled).
template <int N, int L> constexpr int mfma_stages() {
  int s = 0, n = N;
  while (n >= L) {
    n /= L;
    ++s;
  }
  return s;
}
template <int N, int L> constexpr int mfma_rest() {
  int n = N;
  while (n >= L) n /= L;
  return n;
}
// Elements per tile: T = tile / N pencils.
template <int N> constexpr int mfma_tile_elems() { return N >= 4096 ? 4096 : 8192; }
// LDS layout of a tile: element x of pencil q at q * mfma_row + x + x / 32
// (one pad element per 32, so the Stockham writes and the row reads spread
// over the banks), with one more pad element per pencil so that
// consecutive pencils (COL-mode staging) start in different banks.
template <int N> constexpr int mfma_row() { return N + N / 32 + 1; }
template <int N> __device__ __forceinline__ int mfma_lds(int q, int x) {
  return q * mfma_row<N>() + x + (x >> 5);
}
template <int N, int TE = mfma_tile_elems<N>()> constexpr int mfma_buf_elems() {
  return (TE / N) * mfma_row<N>();
}
// Workgroup size: 1024 tile elements per wave, 16 per lane (two waves per
// SIMD for 8192 points).
template <int N, int TE = mfma_tile_elems<N>()> constexpr int mfma_threads() { return TE / 16; }
// Tile elements each lane holds for a stage: 64 / R groups of 16 vectors,
// R / 4 rows of one vector per group.
constexpr int kMfmaRegs = 16;

// Vector (pencil q, butterfly t) of index g of a radix-R stage.  For the
// first stage the load mode's contiguous index runs fastest across lanes
// (ROW: t, COL: q), so the operands come straight from global memory in
// 128-byte runs; later stages use the ROW order.
template <int N, int R, int MODE, int TE = mfma_tile_elems<N>()>
__device__ __forceinline__ void mfma_vec(int g, int& q, int& t) {
  constexpr int stride = N / R;
  constexpr int T = TE / N;
  if constexpr (MODE == MODE_ROW) { q = g / stride; t = g % stride; }
  else { q = g % T; t = g / T; }
}

// Vector index of group gi (of 64 / R) of this lane in a radix-R stage.
template <int R>
__device__ __forceinline__ int mfma_group_vec(int wave, int gi, int lane) {
  return wave * (1024 / R) + gi * 16 + (lane & 15);
}

// First input row of a lane's vector in a radix-R stage: lanes l and
// l + 32 (h = l / 16 and h + 2) hold rows (R / 2) (h & 1) + 0 .. R / 4 - 1
// and the next R / 4 rows.
template <int R>
__device__ __forceinline__ int mfma_first_row(int lane) {
  return (R / 2) * ((lane >> 4) & 1) + (R / 4) * (lane >> 5);
}

// Global -> registers, already in first-stage operand order: lane (wave,
// n, h) of group gi gets rows rb .. rb + R / 4 - 1 (rb = mfma_first_row)
// of its vector in v[gi * R / 4 ..].  Pencils past the end of a ragged last
// tile re-read the last pencil (in bounds, never stored).
template <int N, int R, int LM, int TE = mfma_tile_elems<N>()>
__device__ __forceinline__ void mfma_load(float2 (&v)[kMfmaRegs], const float2* src,
                                          const PassArgs& a, int64_t tile, int tid) {
  constexpr int T = TE / N;
  constexpr int stride = N / R;
  const int lane = tid & 63, wave = tid >> 6;
  const int rb = mfma_first_row<R>(lane);
  // element stride along the pencil: 1 in ROW mode (by construction)
  const int64_t js = LM == MODE_ROW ? 1 : a.ijs;
#pragma unroll
  for (int gi = 0; gi < 64 / R; ++gi) {
    int q, t;
    mfma_vec<N, R, LM, TE>(mfma_group_vec<R>(wave, gi, lane), q, t);
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    const float2* s = src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2) +
                      (int64_t)(t + rb * stride) * js;
    const int64_t step = (int64_t)stride * js;
#pragma unroll
    for (int k = 0; k < R / 4; ++k) v[gi * (R / 4) + k] = s[k * step];
  }
}

// One radix-R leaf for a 16-vector group.  x[k] is row rb + k of the
// lane's vector, already twiddled; lanes l and l + 32 hold the same
// vector's first and second R / 4 rows of the lane group's R / 2 and
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

template <int N, int R, int PREC>
__device__ __forceinline__ void mfma_leaf_store(const float2 (&x)[R / 4],
                                                const LeafA<PREC, R>& A, float2* out,
                                                int64_t pbase, int q, int t, int NS, int lane) {
  const float sgn = mfma_vector_sign(pbase + q, t, NS);
  float xs[R / 2];
#pragma unroll
  for (int k = 0; k < R / 4; ++k) {
    // lane < 32 keeps its real part and gets the partner's; lane >= 32
    // gets the partner's imaginary part and keeps its own
    const auto sw = __builtin_amdgcn_permlane32_swap(
        __builtin_bit_cast(unsigned, x[k].x), __builtin_bit_cast(unsigned, x[k].y), false, false);
    xs[k] = __builtin_bit_cast(float, (unsigned)sw[0]);
    xs[R / 4 + k] = __builtin_bit_cast(float, (unsigned)sw[1]);
  }
  // the four lanes of a vector (l, l ^ 16, l ^ 32, l ^ 48) share (q, t), so
  // the sign needs no exchange
  const int h = lane >> 4;
  const int tm = t & (NS - 1);
  const int base = (t / NS) * NS * R + tm;
  if constexpr (R == 16) {
    f32x4_t yr, yi;
    leaf16<PREC>(A, xs, sgn, yr, yi);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      out[mfma_lds<N>(q, base + (4 * h + i) * NS)] = make_float2(yr[i], yi[i]);
  } else {
    f32x4_t yr[2], yi[2];
    leaf32<PREC>(A, xs, sgn, yr, yi);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[mfma_lds<N>(q, base + (16 * m + 4 * h + i) * NS)] = make_float2(yr[m][i], yi[m][i]);
  }
}

// First stage from the registers mfma_load filled (conjugated for the
// inverse), output to LDS buffer out.
template <int N, int R, int LM, int PREC, int TE = mfma_tile_elems<N>()>
__device__ __forceinline__ void mfma_first_stage(const float2 (&v)[kMfmaRegs], float2* out,
                                                 const LeafA<PREC, R>& A, int conj,
                                                 int64_t pbase, int tid) {
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int gi = 0; gi < 64 / R; ++gi) {
    int q, t;
    mfma_vec<N, R, LM, TE>(mfma_group_vec<R>(wave, gi, lane), q, t);
    float2 x[R / 4];
#pragma unroll
    for (int k = 0; k < R / 4; ++k) {
      x[k] = v[gi * (R / 4) + k];
      if (conj) x[k].y = -x[k].y;
    }
    mfma_leaf_store<N, R, PREC>(x, A, out, pbase, q, t, 1, lane);
  }
}

// Twiddled inputs of one group in a later stage (NS = product of the
// earlier radices): row r of vector (q, t) times w_{NS R}^{(t mod NS) r}.
template <int N, int R>
__device__ __forceinline__ void mfma_stage_inputs(float2 (&x)[R / 4], const float2* in,
                                                  const float2* ltw, int q, int t, int NS,
                                                  int rb) {
  constexpr int stride = N / R;
  const int twstep = N / (NS * R);
  const int tm = t & (NS - 1);
#pragma unroll
  for (int k = 0; k < R / 4; ++k) {
    const int r = rb + k;
    x[k] = cmul(in[mfma_lds<N>(q, t + r * stride)], ltw[tm * r * twstep]);
  }
}

// The one-tile form's later stages, in place in the LDS tile: every lane
// reads the inputs of its groups (twiddled) into registers, the workgroup
// waits, and the leaves write their outputs back to their Stockham places.
// One buffer (not two) leaves room for two workgroups per CU.
template <int N, int R, int PREC, int TE = mfma_tile_elems<N>()>
__device__ __forceinline__ void mfma_later_stages(float2* io, const float2* ltw,
                                                  const LeafA<PREC, R>& A, int64_t pbase,
                                                  int tid) {
  constexpr int S = mfma_stages<N, R>();
  const int lane = tid & 63, wave = tid >> 6;
  const int rb = mfma_first_row<R>(lane);
  int NS = R;
#pragma unroll
  for (int st = 1; st < S; ++st) {
    float2 x[64 / R][R / 4];
#pragma unroll
    for (int gi = 0; gi < 64 / R; ++gi) {
      int q, t;
      mfma_vec<N, R, MODE_ROW, TE>(mfma_group_vec<R>(wave, gi, lane), q, t);
      mfma_stage_inputs<N, R>(x[gi], io, ltw, q, t, NS, rb);
    }
    __syncthreads();  // every input of the stage is read
#pragma unroll
    for (int gi = 0; gi < 64 / R; ++gi) {
      int q, t;
      mfma_vec<N, R, MODE_ROW, TE>(mfma_group_vec<R>(wave, gi, lane), q, t);
      mfma_leaf_store<N, R, PREC>(x[gi], A, io, pbase, q, t, NS, lane);
    }
    __syncthreads();  // every output of the stage is written
    NS *= R;
  }
}

// The persistent form's later stages: ping-pong between two LDS buffers
// (starting from buffer 0; no wait between a stage's reads and its writes,
// and fewer registers held across the waits than in place); returns the
// buffer index holding the result.
template <int N, int R, int PREC>
__device__ __forceinline__ int mfma_later_stages_pingpong(float2 (*buf)[mfma_buf_elems<N>()],
                                                          const float2* ltw,
                                                          const LeafA<PREC, R>& A,
                                                          int64_t pbase, int tid) {
  constexpr int S = mfma_stages<N, R>();
  const int lane = tid & 63, wave = tid >> 6;
  const int rb = mfma_first_row<R>(lane);
  int cur = 0;
  int NS = R;
#pragma unroll
  for (int st = 1; st < S; ++st) {
    const float2* in = buf[cur];
    float2* out = buf[cur ^ 1];
#pragma unroll
    for (int gi = 0; gi < 64 / R; ++gi) {
      int q, t;
      mfma_vec<N, R, MODE_ROW>(mfma_group_vec<R>(wave, gi, lane), q, t);
      float2 x[R / 4];
      mfma_stage_inputs<N, R>(x, in, ltw, q, t, NS, rb);
      mfma_leaf_store<N, R, PREC>(x, A, out, pbase, q, t, NS, lane);
    }
    __syncthreads();
    cur ^= 1;
    NS *= R;
  }
  return cur;
}

// Last step: with a leftover radix, its butterflies read LDS and write
// straight to global memory (lanes ordered by the store mode's contiguous
// index); otherwise the result is copied out in the store mode's order.
template <int N, int SM, int L, int TE = mfma_tile_elems<N>()>
__device__ __forceinline__ void mfma_finish(const float2* res, float2* dst, const float2* ltw,
                                            const PassArgs& a, int64_t tile, int tid) {
  constexpr int T = TE / N;
  constexpr int NTHR = mfma_threads<N, TE>();
  constexpr int REST = mfma_rest<N, L>();
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
    constexpr int EPT = TE / NTHR;
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

// Waves per SIMD the one-tile form asks the compiler for: four (at most
// 128 VGPRs) where two workgroups fit in a CU's LDS, else two.
template <int N, int TE = mfma_tile_elems<N>()> constexpr int mfma_one_tile_waves() {
  return (2 * (mfma_buf_elems<N, TE>() + N) * 8 <= 160 * 1024 || mfma_threads<N, TE>() >= 1024)
             ? 4 : 2;
}

// One tile per workgroup (TE tile elements: the default, or twice that in
// the wide form, whose rotated store writes rows of twice the pencils).
template <int N, int LM, int SM, int PREC, int L, int TE = mfma_tile_elems<N>()>
__global__ void __launch_bounds__((mfma_threads<N, TE>()), (mfma_one_tile_waves<N, TE>()))
fft_pass_mfma(const float2* src, float2* dst, const float2* __restrict__ tw,
              const unsigned short* __restrict__ leaf, const PassArgs a) {
  __shared__ float2 buf[mfma_buf_elems<N, TE>()];
  __shared__ float2 ltw[N];
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  float2 v[kMfmaRegs];
  mfma_load<N, L, LM, TE>(v, src, a, tile, tid);
  for (int i = tid; i < N; i += mfma_threads<N, TE>()) ltw[i] = tw[i];
  LeafA<PREC, L> A;
  A.load(leaf, tid & 63);
  constexpr int T = TE / N;
  mfma_first_stage<N, L, LM, PREC, TE>(v, buf, A, a.conj_in, tile * T, tid);
  __syncthreads();
  mfma_later_stages<N, L, PREC, TE>(buf, ltw, A, tile * T, tid);
  mfma_finish<N, SM, L, TE>(buf, dst, ltw, a, tile, tid);
}

// Persistent form: about one resident workgroup per CU walks the tiles
// (w, w + G, ...; remapped per XCD).  As soon as the first stage has
// consumed the registers, the next tile's loads go out, so they are in
// flight during the remaining stages and the stores.
template <int N, int LM, int SM, int PREC, int L>
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
  mfma_load<N, L, LM>(v, src, a, tile_index(w, ntiles, a.xcd_remap), tid);
  for (int i = tid; i < N; i += mfma_threads<N>()) ltw[i] = tw[i];
  LeafA<PREC, L> A;
  A.load(leaf, tid & 63);
  __syncthreads();  // twiddles in LDS
  while (true) {
    const int64_t tile = tile_index(w, ntiles, a.xcd_remap);
    mfma_first_stage<N, L, LM, PREC>(v, buf[0], A, a.conj_in, tile * T, tid);
    __syncthreads();
    const int64_t wn = w + G;
    // prefetch the next tile (past the end: the last tile again, in bounds)
    mfma_load<N, L, LM>(v, src, a, tile_index(wn < last ? wn : last, ntiles, a.xcd_remap), tid);
    const int cur = mfma_later_stages_pingpong<N, L, PREC>(buf, ltw, A, tile * T, tid);
    mfma_finish<N, SM, L>(buf[cur], dst, ltw, a, tile, tid);
    __syncthreads();  // every read of the result buffer is done
    w = wn;
    if (w >= ntiles) break;
  }
}

template <int N, int LM, int SM, int PREC, int L, int TE = mfma_tile_elems<N>()>
hipError_t launch_mfma(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                       const float2* leaf, hipStream_t stream) {
  constexpr int T = TE / N;
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_pass_mfma<N, LM, SM, PREC, L, TE>), dim3((unsigned)blocks),
                     dim3(mfma_threads<N, TE>()), 0, stream, src, dst, tw,
                     reinterpret_cast<const unsigned short*>(leaf), a);
  return hipGetLastError();
}

template <int N, int LM, int SM, int PREC, int L>
hipError_t launch_mfma_persistent(const PassArgs& a, const float2* src, float2* dst,
                                  const float2* tw, const float2* leaf, hipStream_t stream) {
  constexpr int T = mfma_tile_elems<N>() / N;
  const int64_t tiles = (a.B + T - 1) / T;
  if (tiles <= 0) return hipSuccess;
  static int per_cu = -1;  // resident workgroups per CU for this kernel
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, fft_pass_mfma_persistent<N, LM, SM, PREC, L>, mfma_threads<N>(), 0) !=
        hipSuccess)
      return hipGetLastError();
    per_cu = nb > 0 ? nb : 1;
  }
  int64_t grid = (int64_t)device_cu_count() * per_cu;
  if (grid > tiles) grid = tiles;
  hipLaunchKernelGGL((fft_pass_mfma_persistent<N, LM, SM, PREC, L>), dim3((unsigned)grid),
                     dim3(mfma_threads<N>()), 0, stream, src, dst, tw,
                     reinterpret_cast<const unsigned short*>(leaf), a);
  return hipGetLastError();
}

template <int N, int LM, int SM, int PREC, int PERS, int L>
KernelInfo kernel_info_mfma() {
  static_assert(N >= L && (L == 16 || mfma_rest<N, 32>() < 16), "leaf length");
  constexpr int T = mfma_tile_elems<N>() / N;
  constexpr int LDS = ((PERS ? 2 : 1) * mfma_buf_elems<N>() + N) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(mfma_tile_elems<N>() % (16 * mfma_threads<N>()) == 0, "whole rounds");
  KernelInfo k{N, T, LM, SM, 0, mfma_threads<N>(), LDS,
               PERS ? &launch_mfma_persistent<N, LM, SM, PREC, L>
                    : &launch_mfma<N, LM, SM, PREC, L>,
               PERS, 0, PREC};
  k.mfma_leaf = L;
  return k;
}

// The wide one-tile form (twice the tile elements, one workgroup per CU
// with 1024 threads, four waves per SIMD).
template <int N, int LM, int SM, int PREC, int L>
KernelInfo kernel_info_mfma_wide() {
  constexpr int TE = 2 * mfma_tile_elems<N>();
  constexpr int LDS = (mfma_buf_elems<N, TE>() + N) * 8;
  static_assert(LDS <= 160 * 1024, "tile exceeds LDS");
  static_assert(mfma_threads<N, TE>() <= 1024, "workgroup too large");
  KernelInfo k{N, TE / N, LM, SM, 0, mfma_threads<N, TE>(), LDS,
               &launch_mfma<N, LM, SM, PREC, L, TE>, 0, 0, PREC};
  k.mfma_leaf = L;
  k.mfma_wide = 1;
  return k;
}

template <int N, int PREC, int L>
void add_mfma_kernels_prec(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_COL, PREC, 0, L>());
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_ROW, PREC, 0, L>());
  v.push_back(kernel_info_mfma<N, MODE_COL, MODE_COL, PREC, 0, L>());
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_COL, PREC, 1, L>());
  v.push_back(kernel_info_mfma<N, MODE_ROW, MODE_ROW, PREC, 1, L>());
  v.push_back(kernel_info_mfma<N, MODE_COL, MODE_COL, PREC, 1, L>());
}

// The wide rotate-on-write form of every precision of one length and leaf
// length.
template <int N, int L>
void add_mfma_wide_kernels(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_mfma_wide<N, MODE_ROW, MODE_COL, DFT3D_PREC_BF16X1, L>());
  v.push_back(kernel_info_mfma_wide<N, MODE_ROW, MODE_COL, DFT3D_PREC_FP16X1, L>());
  v.push_back(kernel_info_mfma_wide<N, MODE_ROW, MODE_COL, DFT3D_PREC_BF16X6, L>());
  v.push_back(kernel_info_mfma_wide<N, MODE_ROW, MODE_COL, DFT3D_PREC_BF16X9, L>());
  v.push_back(kernel_info_mfma_wide<N, MODE_ROW, MODE_COL, DFT3D_PREC_FP16X3, L>());
}

// Every precision of one length and leaf length.
template <int N, int L = 16>
void add_mfma_kernels(std::vector<KernelInfo>& v) {
  add_mfma_kernels_prec<N, DFT3D_PREC_BF16X1, L>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_FP16X1, L>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_BF16X6, L>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_BF16X9, L>(v);
  add_mfma_kernels_prec<N, DFT3D_PREC_FP16X3, L>(v);
}

}  // namespace dft3d
