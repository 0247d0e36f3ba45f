// Lengths whose prime factors are all at most 13: one rotate-on-write
// pencil pass whose radix stages run in LDS (the Stockham factorisation of
// eq. (3) with mixed radices 2, 3, 4, 5, 7, 8, 10, 11, 13, 16).
//
// A workgroup of TH threads takes a tile of T pencils (T * NMAX points fit
// in 64 KB of LDS, so two workgroups share a CU; the twiddle table is
// copied next to them where the LDS has room, NMAX <= 2048).  The first
// stage reads its butterflies straight from global memory (lanes along each
// pencil) and writes its outputs to LDS; every later stage reads its
// butterflies' inputs from LDS into registers, waits, transforms and writes
// the outputs back to their Stockham places, and waits again; the finished
// pencils are stored rotated (T consecutive pencils per output row).
//
// Stage s has radix R and ns = the product of the earlier radices.
// Butterfly t (t < n / R) of a pencil takes inputs t + r n / R (r < R),
// multiplies input r by w_{ns R}^{(t mod ns) r}, transforms them with DFT_R
// and writes output r to (t div ns) ns R + (t mod ns) + r ns.  After the
// last stage the pencil is in natural order.  The twiddles come from a
// per-length table (n - 1 entries, FP64-built) holding w_{ns R}^{tm r} at
// (ns - 1) + (r - 1) ns + tm, so that lanes with consecutive tm read
// consecutive entries (conflict-free in LDS).
//
// PassArgs fields used: pencil fields and element strides as for every
// pass, res_mask = n, twp_mask = the radices of the stages, 8 bits each,
// the first stage in the lowest bits (a zero byte ends the list).
#pragma once

#include "pencil_index.h"

namespace dft3d {

// Forward DFT of odd length R in registers, from the pairs x_k + x_{R-k}
// and x_k - x_{R-k}:  y_j = x_0 + sum_k (x_k + x_{R-k}) cos(2 pi j k / R)
// - i sum_k (x_k - x_{R-k}) sin(2 pi j k / R), and y_{R-j} with + i.
template <int R>
__device__ __forceinline__ void dft_odd(float2* x) {
  constexpr int H = (R - 1) / 2;
  float2 s[H], d[H];
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    s[k - 1] = cadd(x[k], x[R - k]);
    d[k - 1] = csub(x[k], x[R - k]);
  }
  float2 y0 = x[0];
#pragma unroll
  for (int k = 0; k < H; ++k) y0 = cadd(y0, s[k]);
  const float2 x0 = x[0];
  static_for<H>([&](auto ji) {
    constexpr int j = decltype(ji)::value + 1;
    float2 a = x0, b = make_float2(0.f, 0.f);
    static_for<H>([&](auto ki) {
      constexpr int k = decltype(ki)::value + 1;
      constexpr CosSin cs = unit_angle((long)j * k, R);
      constexpr float c = (float)cs.c, sn = (float)cs.s;
      a.x += s[k - 1].x * c;
      a.y += s[k - 1].y * c;
      b.x += d[k - 1].x * sn;
      b.y += d[k - 1].y * sn;
    });
    x[j] = make_float2(a.x + b.y, a.y - b.x);      // a - i b
    x[R - j] = make_float2(a.x - b.y, a.y + b.x);  // a + i b
  });
  x[0] = y0;
}

constexpr int smallest_factor(int r) {
  for (int f = 2; f * f <= r; ++f)
    if (r % f == 0) return f;
  return r;
}

// Forward DFT of length R in registers: powers of two and odd primes
// directly; other R = A B (A its smallest prime factor) by the four-step
// identity of eq. (3) in registers: DFT_A over a for every b (input index
// b + B a), twiddle w_R^{b a'}, DFT_B over b (output index a' + A b').
template <int R>
__device__ __forceinline__ void dft_mixed(float2* x) {
  if constexpr ((R & (R - 1)) == 0) {
    dft<R>(x);
  } else if constexpr (smallest_factor(R) == R) {
    dft_odd<R>(x);
  } else {
    constexpr int A = smallest_factor(R), B = R / A;
    float2 z[R];
    static_for<B>([&](auto bi) {
      constexpr int b = decltype(bi)::value;
      float2 s[A];
#pragma unroll
      for (int a = 0; a < A; ++a) s[a] = x[b + B * a];
      dft_mixed<A>(s);
      static_for<A>([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        z[b + B * a] = mul_root<b * a, R>(s[a]);
      });
    });
#pragma unroll
    for (int a = 0; a < A; ++a) {
      float2 s[B];
#pragma unroll
      for (int b = 0; b < B; ++b) s[b] = z[b + B * a];
      dft_mixed<B>(s);
#pragma unroll
      for (int b = 0; b < B; ++b) x[a + A * b] = s[b];
    }
  }
}

// Calls f(std::integral_constant<int, R>) for a stage radix R the kernel
// variant runs: the primes 2, 3, 5, 7 and 4, 8 always; with COMP also the
// composites 10 and 16 (variant 1 up to NMAX = 2048, where they keep the
// kernel at 128 VGPRs or fewer); with VAR 2 also 11 and 13.  The host
// encodes no other radix for the kernel it picks.
template <int VAR, bool COMP, class F>
__device__ __forceinline__ void with_radix(int R, F&& f) {
  switch (R) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 10:
      if constexpr (COMP) f(std::integral_constant<int, 10>{});
      break;
    case 16:
      if constexpr (COMP) f(std::integral_constant<int, 16>{});
      break;
    case 11:
      if constexpr (VAR >= 2) f(std::integral_constant<int, 11>{});
      break;
    case 13:
      if constexpr (VAR >= 2) f(std::integral_constant<int, 13>{});
      break;
    default: break;
  }
}

// One radix-R stage over pencil q (pen = its LDS row, n points): thread p
// of the P threads of the pencil runs butterflies t = p, p + P, ... (at most
// K = ceil(V / R) of them, V = NMAX / P).
template <int R, int V>
__device__ __forceinline__ void mixed_stage(float2* pen, int n, int ns,
                                            const float2* __restrict__ tw, int p, int P) {
  constexpr int K = (V + R - 1) / R;
  const int nr = n / R;
  const int dq = P / ns, dr = P - dq * ns;
  int g = p / ns, tm = p - g * ns;  // t div ns, t mod ns for t = p
  float2 a[K][R];
  int ob[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int t = p + P * i;
    ob[i] = g * ns * R + tm;
    if (t < nr) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[i][r] = pen[t + r * nr];
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) a[i][r] = cmul(a[i][r], tw[(ns - 1) + (r - 1) * ns + tm]);
      }
      dft_mixed<R>(a[i]);
    }
    tm += dr;
    g += dq;
    if (tm >= ns) {
      tm -= ns;
      ++g;
    }
  }
  __syncthreads();  // every input of the stage is read
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (p + P * i < nr) {
#pragma unroll
      for (int r = 0; r < R; ++r) pen[ob[i] + r * ns] = a[i][r];
    }
  }
  __syncthreads();  // every output of the stage is written
}

// The first stage (ns = 1) straight from global memory: butterfly t reads
// the pencil's points t + r n / R (consecutive t on consecutive lanes),
// all of the thread's loads in flight before the transforms, and writes
// its outputs to t R + r in LDS; no twiddles.
template <int R, int V, int K = (V + R - 1) / R>
__device__ __forceinline__ void mixed_first_load(float2 (&a)[K][R], const float2* s,
                                                 int64_t ijs, int n, int p, int P) {
  const int nr = n / R;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int t = p + P * i;
    if (t < nr) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[i][r] = s[(int64_t)(t + r * nr) * ijs];
    }
  }
}

template <int R, int V, int K = (V + R - 1) / R>
__device__ __forceinline__ void mixed_first_compute(float2 (&a)[K][R], int conj, float2* pen,
                                                    int n, int p, int P) {
  const int nr = n / R;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int t = p + P * i;
    if (t < nr) {
      if (conj) {
#pragma unroll
        for (int r = 0; r < R; ++r) a[i][r].y = -a[i][r].y;
      }
      dft_mixed<R>(a[i]);
#pragma unroll
      for (int r = 0; r < R; ++r) pen[t * R + r] = a[i][r];
    }
  }
  __syncthreads();  // every output of the stage is written
}

template <int R, int V>
__device__ __forceinline__ void mixed_first_stage(const float2* s, int64_t ijs, int conj,
                                                  float2* pen, int n, int p, int P) {
  float2 a[(V + R - 1) / R][R];
  mixed_first_load<R, V>(a, s, ijs, n, p, P);
  mixed_first_compute<R, V>(a, conj, pen, n, p, P);
}

// The later stages (radices in code, ns = the first radix) and the store
// of the tile's pencils: COL (rotated: consecutive pencils contiguous)
// with the thread on pencil tid mod T and outputs k = tid / T + (TH / T) i,
// so lanes run across the pencils; ROW (the pencil's own points
// contiguous) with the thread on pencil tid / P and outputs k = p + P i, so
// lanes run along the pencil.
template <int T, int NMAX, int TH, int VAR, int SM = MODE_COL>
__device__ __forceinline__ void mixed_rest(uint64_t code, int ns, float2* buf, float2* pen,
                                           const float2* twv, float2* dst, const PassArgs& a,
                                           int64_t tile, int n, int sq, int tid, int p) {
  constexpr int P = TH / T;
  constexpr int V = NMAX / P;
  constexpr bool COMP = VAR == 1 && NMAX <= 2048;  // radices 10 and 16
  while (code) {
    const int R = (int)(code & 255);
    code >>= 8;
    with_radix<VAR, COMP>(R, [&](auto rc) {
      mixed_stage<decltype(rc)::value, V>(pen, n, ns, twv, p, P);
    });
    ns *= R;
  }
  if constexpr (SM == MODE_ROW) {
    const int q = tid / P;
    const int64_t b = tile * T + q;
    if (b < a.B) {
      float2* d = dst + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int k = p + P * i;
        if (k < n) {
          float2 w = pen[k];
          if (a.conj_out) w.y = -w.y;
          d[k * a.oks] = w;
        }
      }
    }
    return;
  }
  const int qs = tid % T;
  const int64_t b = tile * T + qs;
  if (b < a.B) {
    float2* d = dst + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);
    const float2* ps = buf + qs * sq;
    constexpr int S = T * NMAX / TH;  // outputs per thread, at most
    constexpr int KS = TH / T;
    float2 w[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int k = tid / T + KS * i;
      if (k < n) w[i] = ps[k];
    }
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int k = tid / T + KS * i;
      if (k < n) {
        if (a.conj_out) w[i].y = -w[i].y;
        d[k * a.oks] = w[i];
      }
    }
  }
}

// VAR: 1 without the radix-11 and radix-13 stages (whose registers would
// lower the occupancy of every other stage too), 2 with them.  LM, SM: the
// load and store modes.  ROW loads run the first stage straight from
// global memory (lanes along each pencil); COL loads (consecutive pencils
// contiguous, the pencil's points at stride ijs) first copy the tile into
// LDS with lanes across the pencils (thread on pencil tid mod T), then run
// the first stage from there.
template <int T, int NMAX, int TH, int VAR, int LM = MODE_ROW, int SM = MODE_COL>
__global__ void __launch_bounds__(TH)
fft_mixed_kernel(const float2* src, float2* dst, const float2* __restrict__ tw,
                 const float2* __restrict__ twp, const PassArgs a) {
  constexpr int P = TH / T;             // threads per pencil
  constexpr int V = NMAX / P;           // points per thread
  constexpr bool COMP = VAR == 1 && NMAX <= 2048;  // radices 10 and 16
  // twiddle table in LDS where two workgroups per CU still fit
  constexpr bool TWL = 2 * (T * NMAX + NMAX) * 8 <= 160 * 1024;
  __shared__ float2 buf[T * NMAX + (TWL ? NMAX : 0)];
  const int n = (int)a.res_mask;  // n < NMAX (NMAX is a power of two, n is not)
  const int sq = n + 1;           // LDS pencil stride; T sq <= T NMAX
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  const int q = tid / P, p = tid % P;
  float2* pen = buf + q * sq;
  const float2* twv = TWL ? buf + T * NMAX : tw;
  if constexpr (TWL) {  // the twiddle table's n - 1 entries into LDS
    float2* tl = buf + T * NMAX;
#pragma unroll
    for (int i = 0; i < (NMAX + TH - 1) / TH; ++i) {
      const int j = tid + TH * i;
      if (j < n - 1) tl[j] = tw[j];
    }
  }
  uint64_t code = (uint64_t)a.twp_mask;
  int ns;
  if constexpr (LM == MODE_COL) {
    {  // the tile into LDS, lanes across the pencils
      const int qs = tid % T;
      int64_t b = tile * T + qs;
      b = b < a.B ? b : a.B - 1;
      const float2* s =
          src + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
      float2* ps = buf + qs * sq;
      constexpr int KS = TH / T;
#pragma unroll
      for (int i = 0; i < NMAX / KS; ++i) {
        const int k = tid / T + KS * i;
        if (k < n) ps[k] = s[(int64_t)k * a.ijs];
      }
    }
    __syncthreads();  // the tile is in LDS
    const int R = (int)(code & 255);
    code >>= 8;
    with_radix<VAR, COMP>(R, [&](auto rc) {
      constexpr int RR = decltype(rc)::value;
      float2 v[(V + RR - 1) / RR][RR];
      mixed_first_load<RR, V>(v, pen, 1, n, p, P);
      __syncthreads();  // every input of the first stage is read
      mixed_first_compute<RR, V>(v, a.conj_in, pen, n, p, P);
    });
    ns = R;
  } else {
    // pencils past the end of a ragged last tile read the last pencil
    int64_t b = tile * T + q;
    b = b < a.B ? b : a.B - 1;
    const float2* s = src + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
    const int R = (int)(code & 255);
    code >>= 8;
    with_radix<VAR, COMP>(R, [&](auto rc) {
      mixed_first_stage<decltype(rc)::value, V>(s, a.ijs, a.conj_in, pen, n, p, P);
    });
    ns = R;
  }
  mixed_rest<T, NMAX, TH, VAR, SM>(code, ns, buf, pen, twv, dst, a, tile, n, sq, tid, p);
}

// Stages of a compile-time radix code (the first stage done, NS = its radix).
template <uint64_t CODE, int NS, int V, int N>
__device__ __forceinline__ void mixed_stages_fixed(float2* pen, const float2* twv, int p,
                                                   int P) {
  if constexpr (CODE != 0) {
    constexpr int R = (int)(CODE & 255);
    mixed_stage<R, V>(pen, N, NS, twv, p, P);
    mixed_stages_fixed<(CODE >> 8), NS * R, V, N>(pen, twv, p, P);
  }
}

// The same pass for one length N known at compile time, with its radix code
// CODE (variant 1 radices): the stage sizes, the butterfly index arithmetic
// and the LDS offsets fold into constants and the radix switch disappears.
template <int T, int NMAX, int TH, int N, uint64_t CODE>
__global__ void __launch_bounds__(TH)
fft_mixed_fixed(const float2* src, float2* dst, const float2* __restrict__ tw,
                const float2* __restrict__ twp, const PassArgs a) {
  constexpr int P = TH / T;
  constexpr int V = NMAX / P;
  constexpr bool TWL = 2 * (T * NMAX + NMAX) * 8 <= 160 * 1024;
  static_assert(N < NMAX, "length fits the tile");
  __shared__ float2 buf[T * NMAX + (TWL ? NMAX : 0)];
  constexpr int sq = N + 1;
  const int tid = threadIdx.x;
  const int64_t tile = tile_index(blockIdx.x, gridDim.x, a.xcd_remap);
  const int q = tid / P, p = tid % P;
  float2* pen = buf + q * sq;
  const float2* twv = TWL ? buf + T * NMAX : tw;
  if constexpr (TWL) {
    float2* tl = buf + T * NMAX;
#pragma unroll
    for (int i = 0; i < (NMAX + TH - 1) / TH; ++i) {
      const int j = tid + TH * i;
      if (j < N - 1) tl[j] = tw[j];
    }
  }
  int64_t b = tile * T + q;
  b = b < a.B ? b : a.B - 1;
  const float2* s = src + pencil_offset_any(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
  constexpr int R1 = (int)(CODE & 255);
  mixed_first_stage<R1, V>(s, a.ijs, a.conj_in, pen, N, p, P);
  mixed_stages_fixed<(CODE >> 8), R1, V, N>(pen, twv, p, P);
  mixed_rest<T, NMAX, TH, 1>(0, N, buf, pen, twv, dst, a, tile, N, sq, tid, p);  // store
}

template <int T, int NMAX, int TH, int N, uint64_t CODE>
hipError_t launch_mixed_fixed(const PassArgs& a, const float2* src, float2* dst,
                              const float2* tw, const float2* twp, hipStream_t stream) {
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (a.res_mask != N || (uint64_t)a.twp_mask != CODE) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fft_mixed_fixed<T, NMAX, TH, N, CODE>), dim3((unsigned)blocks), dim3(TH),
                     0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

// The compiled-length kernel reads pencils along their points and stores
// across the pencils (the rotating pass); the registry also offers it for
// the in-layout passes (the pass arguments carry the strides).
template <int T, int NMAX, int TH, int N, uint64_t CODE>
KernelInfo kernel_info_mixed_fixed() {
  constexpr int LDS = (T * NMAX + (2 * (T * NMAX + NMAX) * 8 <= 160 * 1024 ? NMAX : 0)) * 8;
  static_assert(2 * LDS <= 160 * 1024, "two workgroups per CU");
  KernelInfo k{NMAX, T, MODE_ROW, MODE_COL, 0, TH, LDS, &launch_mixed_fixed<T, NMAX, TH, N, CODE>,
               0, 0};
  k.mixed = 1;
  k.fixed_n = N;
  k.fixed_code = CODE;
  return k;
}

template <int T, int NMAX, int TH, int VAR, int LM = MODE_ROW, int SM = MODE_COL>
hipError_t launch_mixed(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                        const float2* twp, hipStream_t stream) {
  const int64_t blocks = (a.B + T - 1) / T;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (a.res_mask < 2 || a.res_mask >= NMAX || !mixed_kernel_runs(VAR, NMAX, (uint64_t)a.twp_mask))
    return hipErrorInvalidValue;  // a stage radix this kernel does not run
  hipLaunchKernelGGL((fft_mixed_kernel<T, NMAX, TH, VAR, LM, SM>), dim3((unsigned)blocks),
                     dim3(TH), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int T, int NMAX, int TH, int VAR, int LM = MODE_ROW, int SM = MODE_COL>
KernelInfo kernel_info_mixed() {
  constexpr int LDS = (T * NMAX + (2 * (T * NMAX + NMAX) * 8 <= 160 * 1024 ? NMAX : 0)) * 8;
  static_assert(2 * LDS <= 160 * 1024, "two workgroups per CU");
  static_assert(TH % T == 0 && NMAX % (TH / T) == 0 && TH <= 1024, "tile shape");
  KernelInfo k{NMAX, T, LM, SM, 0, TH, LDS, &launch_mixed<T, NMAX, TH, VAR, LM, SM>, 0, 0};
  k.mixed = VAR;
  return k;
}

}  // namespace dft3d
