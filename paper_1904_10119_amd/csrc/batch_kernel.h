// Batched form: many 3D DFTs of different shapes in a few launches.
//
// Every (problem, pass) of a batch becomes a work item; the tiles of all
// items of one pass level are laid out consecutively, and one launch of
// batch_level_kernel runs a whole level (one workgroup per tile, the tile's
// item found by binary search).  Fused plane passes (slab) are items of
// their own kind, one workgroup per plane, run by batch_plane_level_kernel
// in a launch of their own for the level.  The kernel boundary between levels orders
// each pass of a problem after the previous one, so there are no waits
// between workgroups: three launches run 96 pencil-schedule problems.
//
// batch_persistent_kernel (one launch for all levels, tiles taken from an
// atomic queue with per-item completion counters) is kept for study but is
// not used: on MI355X its first runs did not complete (see the design
// notes), and it stays switched off until the cause is shown.
#pragma once

#include "pass_kernel.h"
#include "plane_kernel.h"

namespace dft3d {

// Workgroup size of the batched kernel; tile = kBatchThreads / P(n) pencils.
constexpr int kBatchThreads = 256;
// Longest transform length a batched item may have.
constexpr int kBatchMaxN = 256;

template <int N> constexpr int batch_tile() {
  return kBatchThreads / (N / Blocking<N>::E);
}

struct BatchItem {
  PassArgs a;         // pencil decomposition and strides of the pass
  const float2* src;  // refreshed on every call
  float2* dst;
  const float2* tw;   // root table of length n
  const float2* twp;  // plane items: root table of length n1
  int64_t first;      // queue position of the item's first tile
  int64_t ntiles;     // tiles, or planes for plane items
  int32_t n;          // transform length (plane items: row length n2)
  int32_t n1;         // plane items: column length; 0 for 1D passes
  int32_t dep;        // item whose completion this one waits for, -1: none
  int32_t lmode, smode;
};

// Fused plane passes the batched plane kernel runs: (n1, n2) planes with
// both sides in {32, 64, 128}, n1 n2 / 256 elements per thread.
__host__ __device__ constexpr bool batch_plane_shape(int n1, int n2) {
  return (n1 == 32 || n1 == 64 || n1 == 128) && (n2 == 32 || n2 == 64 || n2 == 128);
}

struct BatchState {  // zeroed before every launch
  unsigned long long head;  // next ticket
  unsigned int error;       // set when a bounded wait runs out
  unsigned int pad;
};

// LDS bytes of the largest tile the batched kernel runs.
template <int N> constexpr int batch_lds_elems() {
  return num_stages<Blocking<N>>() > 1 ? batch_tile<N>() * lds_pencil_stride<N, batch_tile<N>()>()
                                       : 1;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kBatchLdsElems =
    cmax(cmax(cmax(batch_lds_elems<256>(), batch_lds_elems<128>()), batch_lds_elems<64>()),
         cmax(batch_lds_elems<32>(), batch_lds_elems<16>()));

template <int N, int LM, int SM>
__device__ __forceinline__ void batch_tile_run(const BatchItem& it, int64_t tile, float2* lds) {
  using BL = Blocking<N>;
  constexpr int E = BL::E;
  constexpr int P = N / E;
  constexpr int T = batch_tile<N>();
  constexpr int NST = num_stages<BL>();
  constexpr int SQ = lds_pencil_stride<N, T>();
  const int tid = threadIdx.x;
  int q, p;
  thread_map<(NST > 1 ? LM : SM), T, P>(tid, q, p);
  float2 v[E];
  load_tile<N, T, E, P, LM, 0>(v, it.src, it.a, tile, q, p);
  transform_store_tile<N, BL, T, LM, SM, 0, 0, E, P, SQ>(v, it.dst, it.tw, nullptr, lds, it.a,
                                                         tile, tid, q, p);
}

template <int N>
__device__ __forceinline__ void batch_tile_modes(const BatchItem& it, int64_t tile,
                                                 float2* lds) {
  if (it.lmode == MODE_ROW && it.smode == MODE_COL)
    batch_tile_run<N, MODE_ROW, MODE_COL>(it, tile, lds);
  else if (it.lmode == MODE_ROW)
    batch_tile_run<N, MODE_ROW, MODE_ROW>(it, tile, lds);
  else
    batch_tile_run<N, MODE_COL, MODE_COL>(it, tile, lds);
}

// Relaxed device-scope load: reads the coherent value without the L2
// invalidate that an acquire performs, so polling does not disturb the
// caches of the workgroups being waited for.
__device__ __forceinline__ unsigned int load_relaxed(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup per tile of the items [item_lo, item_hi) of one level; tile
// t of the launch belongs to the last item whose first tile is <= t + base.
__global__ void __launch_bounds__(kBatchThreads)
batch_level_kernel(const BatchItem* __restrict__ items, int item_lo, int item_hi,
                   int64_t base) {
  __shared__ float2 lds[kBatchLdsElems];
  const int64_t ticket = base + blockIdx.x;
  int lo = item_lo, hi = item_hi - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= ticket) lo = mid; else hi = mid - 1;
  }
  const BatchItem& it = items[lo];
  const int64_t tile = ticket - it.first;
  switch (it.n) {
    case 1: batch_tile_modes<1>(it, tile, lds); break;
    case 2: batch_tile_modes<2>(it, tile, lds); break;
    case 4: batch_tile_modes<4>(it, tile, lds); break;
    case 8: batch_tile_modes<8>(it, tile, lds); break;
    case 16: batch_tile_modes<16>(it, tile, lds); break;
    case 32: batch_tile_modes<32>(it, tile, lds); break;
    case 64: batch_tile_modes<64>(it, tile, lds); break;
    case 128: batch_tile_modes<128>(it, tile, lds); break;
    default: batch_tile_modes<256>(it, tile, lds); break;
  }
}

// Planes of at most this many points run in the small-plane launch (about
// 35 KB of LDS, several workgroups per CU); larger ones in the large-plane
// launch (136 KB, one workgroup per CU).
constexpr int kBatchSmallPlane = 4096;

// Threads of a plane workgroup: 256 for small planes, 1024 for large ones.
template <int LARGE> constexpr int batch_plane_threads() { return LARGE ? 1024 : 256; }

// One workgroup per plane of the plane items [item_lo, item_hi) of one
// level (fused 2D DFT of the plane, as fft_plane_kernel).  LARGE selects
// the plane shapes above kBatchSmallPlane points.
template <int LARGE>
__global__ void __launch_bounds__(batch_plane_threads<LARGE>())
batch_plane_level_kernel(const BatchItem* __restrict__ items, int item_lo, int item_hi,
                         int64_t base) {
  __shared__ float2 lds[LARGE ? plane_lds_elems<128, 128>() : plane_lds_elems<128, 32>()];
  const int64_t ticket = base + blockIdx.x;
  int lo = item_lo, hi = item_hi - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= ticket) lo = mid; else hi = mid - 1;
  }
  const BatchItem& it = items[lo];
  const int64_t plane = ticket - it.first;
  const int tid = threadIdx.x;
#define DFT3D_PLANE_CASE(A, B)                                                              \
  if (it.n1 == A && it.n == B) {                                                            \
    plane_run<A, B, A * B / batch_plane_threads<LARGE>()>(it.src, it.dst, it.tw, it.twp,     \
                                                         it.a, plane, lds, tid);           \
    return;                                                                                 \
  }
  if constexpr (!LARGE) {
    static_assert(plane_lds_elems<128, 32>() >= plane_lds_elems<32, 128>() &&
                      plane_lds_elems<128, 32>() >= plane_lds_elems<64, 64>(),
                  "small-plane LDS");
    DFT3D_PLANE_CASE(32, 32)
    DFT3D_PLANE_CASE(32, 64)
    DFT3D_PLANE_CASE(32, 128)
    DFT3D_PLANE_CASE(64, 32)
    DFT3D_PLANE_CASE(64, 64)
    DFT3D_PLANE_CASE(128, 32)
  } else {
    DFT3D_PLANE_CASE(64, 128)
    DFT3D_PLANE_CASE(128, 64)
    DFT3D_PLANE_CASE(128, 128)
  }
#undef DFT3D_PLANE_CASE
}

__global__ void __launch_bounds__(kBatchThreads)
batch_zero_kernel(BatchState* st, unsigned int* done, int nitems) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    st->head = 0;
    st->error = 0;
  }
  for (int j = i; j < nitems; j += gridDim.x * blockDim.x) done[j] = 0;
}

__global__ void __launch_bounds__(kBatchThreads)
batch_persistent_kernel(const BatchItem* __restrict__ items, int nitems, int64_t total,
                        BatchState* st, unsigned int* done, unsigned int spin_limit) {
  __shared__ float2 lds[kBatchLdsElems];
  __shared__ long long s_ticket;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  while (true) {
    if (tid == 0) {
      const unsigned long long t =
          __hip_atomic_fetch_add(&st->head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      long long ticket = (long long)t;
      int item = -1;
      if (ticket < total) {
        // last item whose first tile is at or before the ticket
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (items[mid].first <= ticket) lo = mid; else hi = mid - 1;
        }
        item = lo;
        const int dep = items[item].dep;
        if (dep >= 0) {
          const unsigned int need = (unsigned int)items[dep].ntiles;
          unsigned int spins = 0;
          while (load_relaxed(&done[dep]) < need) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins >= spin_limit) {  // never expected; stay hang-free
              __hip_atomic_fetch_or(&st->error, 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
          }
          // one acquire per satisfied wait: the producers' stores become
          // visible here, and the barrier below extends that to every wave
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      s_ticket = ticket;
      s_item = item;
    }
    __syncthreads();
    const long long ticket = s_ticket;
    const int item = s_item;
    if (ticket >= total) break;
    const BatchItem& it = items[item];
    const int64_t tile = ticket - it.first;
    switch (it.n) {
      case 1: batch_tile_modes<1>(it, tile, lds); break;
      case 2: batch_tile_modes<2>(it, tile, lds); break;
      case 4: batch_tile_modes<4>(it, tile, lds); break;
      case 8: batch_tile_modes<8>(it, tile, lds); break;
      case 16: batch_tile_modes<16>(it, tile, lds); break;
      case 32: batch_tile_modes<32>(it, tile, lds); break;
      case 64: batch_tile_modes<64>(it, tile, lds); break;
      case 128: batch_tile_modes<128>(it, tile, lds); break;
      default: batch_tile_modes<256>(it, tile, lds); break;
    }
    // every wave's stores complete and visible device-wide before the tile
    // is counted
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0)
      __hip_atomic_fetch_add(&done[item], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace dft3d
