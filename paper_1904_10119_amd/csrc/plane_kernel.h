// Fused 2D DFT of whole (n1, n2) planes, one plane per workgroup: the first
// half of the slab schedule (eq. (6), Fig. 5) in one HBM pass.  The rows are
// transformed in registers and LDS as in the pass kernels, the row results
// stay in LDS as the plane, and the columns are read from there, transformed
// and stored; only planes of up to 2^14 points (128 KB) qualify.
//
// The plane is contiguous: element (i1, i2) of plane b sits at
// b2*is2 + b1*is1 + b0*is0 + i1*n2 + i2 (pencil-index fields as in PassArgs)
// on input and with the output strides on output.
#pragma once

#include "pass_kernel.h"

namespace dft3d {

// Radices of a length-N transform with E elements per thread (E <= N,
// both powers of two): E, then min(E, N / E), then the rest.
template <int N, int E_> struct PlaneBlocking {
  static_assert(E_ <= N, "at most N elements per thread");
  static constexpr int E = E_;
  static constexpr int R0 = E_;
  static constexpr int R1 = (N / E_) < E_ ? (N / E_) : E_;
  static constexpr int R2 = N / (E_ * R1);
  static_assert(R2 <= E_, "three stages at most");
};

// Elements per thread for an n1 x n2 plane: workgroups of at most 1024.
template <int N1, int N2> constexpr int plane_elems() { return N1 * N2 <= 8192 ? 8 : 16; }

// Radix stages of T length-N pencils held as v (thread (q, p) has elements
// p + P e), with LDS exchanges (pencil stride SQ) between them; the last
// exchange maps threads to LAST_MODE.  On return v[e] is output p + P e.
// The caller makes sure no thread still reads lds when this starts.
template <int N, class BL, int T, int SQ, int LAST_MODE>
__device__ __forceinline__ void plane_stages(float2 (&v)[BL::E], float2* lds,
                                             const float2* tw, int tid, int& q, int& p) {
  constexpr int E = BL::E, P = N / E, NST = num_stages<BL>();
  radix_stage<N, E, P, 1, BL::R0>(v, p, tw);
  if constexpr (NST == 2) {
    lds_exchange<N, E, P, T, SQ, 1, BL::R0, LAST_MODE>(v, lds, tid, q, p);
    radix_stage<N, E, P, BL::R0, BL::R1>(v, p, tw);
  } else if constexpr (NST == 3) {
    lds_exchange<N, E, P, T, SQ, 1, BL::R0, MODE_ROW>(v, lds, tid, q, p);
    radix_stage<N, E, P, BL::R0, BL::R1>(v, p, tw);
    __syncthreads();  // every read of the first exchange is done
    lds_exchange<N, E, P, T, SQ, BL::R0, BL::R1, LAST_MODE>(v, lds, tid, q, p);
    radix_stage<N, E, P, BL::R0 * BL::R1, BL::R2>(v, p, tw);
  }
}

// LDS pencil stride: one pad element per 32 plus one, an odd multiple of
// 8 bytes, so a wavefront across pencils spreads over the banks and the
// largest plane (128 x 128) fits.
template <int N> constexpr int plane_stride() { return N + N / 32 + 1; }
template <int N1, int N2> constexpr int plane_lds_elems() {
  constexpr int a = N1 * plane_stride<N2>();
  constexpr int b = N2 * plane_stride<N1>();
  return a > b ? a : b;
}

// 2D DFT of plane b with E elements per thread (N1 * N2 / E threads).
// tw2: roots of length n2 (rows), tw1: roots of length n1 (columns).
template <int N1, int N2, int E>
__device__ __forceinline__ void plane_run(const float2* src, float2* dst,
                                          const float2* __restrict__ tw2,
                                          const float2* __restrict__ tw1, const PassArgs& a,
                                          int64_t b, float2* lds, int tid) {
  using BR = PlaneBlocking<N2, E>;
  using BC = PlaneBlocking<N1, E>;
  constexpr int P2 = N2 / E, P1 = N1 / E;
  constexpr int SQR = plane_stride<N2>();  // row pencils; also the plane rows
  constexpr int SQC = plane_stride<N1>();  // column pencils
  const float2* s = src + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.is0, a.is1, a.is2);
  float2* d = dst + pencil_offset(b, a.m0, a.m1, a.s0, a.s1, a.os0, a.os1, a.os2);

  // rows: thread (q, p) holds elements p + P2 e of row q
  int q, p;
  thread_map<MODE_ROW, N1, P2>(tid, q, p);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = s[q * N2 + p + P2 * e];
    if (a.conj_in) v[e].y = -v[e].y;
  }
  plane_stages<N2, BR, N1, SQR, MODE_ROW>(v, lds, tw2, tid, q, p);
  __syncthreads();  // the row exchanges' reads are done
#pragma unroll
  for (int e = 0; e < E; ++e) lds[q * SQR + lds_pad_index(p + P2 * e)] = v[e];
  __syncthreads();

  // columns: thread (q, p) holds elements p + P1 e of column q, consecutive
  // threads on consecutive columns so that the stores are contiguous
  thread_map<MODE_COL, N2, P1>(tid, q, p);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = lds[(p + P1 * e) * SQR + lds_pad_index(q)];
  if constexpr (num_stages<BC>() > 1) __syncthreads();  // plane read before reuse
  plane_stages<N1, BC, N2, SQC, MODE_COL>(v, lds, tw1, tid, q, p);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    float2 o = v[e];
    if (a.conj_out) o.y = -o.y;
    d[(p + P1 * e) * N2 + q] = o;
  }
}

template <int N1, int N2>
__global__ void __launch_bounds__((N1 * N2 / plane_elems<N1, N2>()))
fft_plane_kernel(const float2* src, float2* dst, const float2* __restrict__ tw2,
                 const float2* __restrict__ tw1, const PassArgs a) {
  __shared__ float2 lds[plane_lds_elems<N1, N2>()];
  plane_run<N1, N2, plane_elems<N1, N2>()>(src, dst, tw2, tw1, a, blockIdx.x, lds,
                                           threadIdx.x);
}

template <int N1, int N2>
hipError_t launch_plane(const PassArgs& a, const float2* src, float2* dst, const float2* tw,
                        const float2* twp, hipStream_t stream) {
  if (a.B <= 0) return hipSuccess;
  if (a.B > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fft_plane_kernel<N1, N2>), dim3((unsigned)a.B),
                     dim3(N1 * N2 / plane_elems<N1, N2>()), 0, stream, src, dst, tw, twp, a);
  return hipGetLastError();
}

template <int N1, int N2>
KernelInfo kernel_info_plane() {
  constexpr int LDS = plane_lds_elems<N1, N2>() * 8;
  static_assert(LDS <= 160 * 1024, "plane exceeds LDS");
  KernelInfo k{N2, 1, MODE_ROW, MODE_ROW, 0, N1 * N2 / plane_elems<N1, N2>(), LDS,
               &launch_plane<N1, N2>, 0, 0, 0};
  k.plane_rows = N1;
  return k;
}

}  // namespace dft3d
