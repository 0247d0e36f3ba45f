// Batched form: many 3D DFTs of different shapes in a few launches, or in
// one.
//
// Every (problem, pass) of a batch becomes a work item; the tiles of all
// items of one pass level are laid out consecutively (level-major order).
//
// Level launches: one launch of batch_level_kernel runs a whole level (one
// workgroup per tile, the tile's item found by binary search).  Fused plane
// passes (slab) are items of their own kind, one workgroup per plane, run by
// batch_plane_level_kernel in a launch of their own for the level.  The
// kernel boundary between levels orders each pass of a problem after the
// previous one.
//
// One persistent launch: batch_persistent_kernel runs every level.  Resident
// workgroups take tickets (tile numbers in level-major order) from a device
// counter; before a tile of pass k of a problem runs, the workgroup waits
// until every tile of pass k - 1 of that problem has been counted done.
// Those tiles have smaller tickets, so the holder of the smallest unfinished
// ticket never waits and the launch always drains, whatever number of
// workgroups is resident.  Waits are bounded (a poll limit, after which the
// workgroup flags an error and goes on), so a broken descriptor table cannot
// hang the device.
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

// Counters of the persistent launch.  Zero before the first launch (the
// host clears them once); the last workgroup to leave a launch zeroes head,
// exited and every done[] counter again, so launches and graph replays need
// no reset in between.  error is sticky (cleared by the host when it reads
// it).
struct BatchState {
  unsigned long long head;  // next ticket
  unsigned int exited;      // workgroups that have left the ticket loop
  unsigned int error;       // set when a bounded wait runs out
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

// LDS of the persistent kernel: the largest 1D tile or small plane.
constexpr int kBatchPersistentLds = cmax(kBatchLdsElems, plane_lds_elems<128, 32>());

// Plane shapes the persistent kernel runs (small planes, 256 threads).
__host__ __device__ constexpr bool batch_persistent_plane_shape(int n1, int n2) {
  return batch_plane_shape(n1, n2) && n1 * n2 <= kBatchSmallPlane;
}

// The item a ticket belongs to: the last of [lo, hi) whose first tile is at
// or before it.
__device__ __forceinline__ int batch_find_item(const BatchItem* items, int lo, int hi,
                                               int64_t ticket) {
  hi -= 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= ticket) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One small-plane item tile (a whole plane) on 256 threads.
__device__ __noinline__ void batch_small_plane(const BatchItem& it, int64_t plane,
                                                  float2* lds, int tid) {
#define DFT3D_PLANE_CASE(A, B)                                                               \
  if (it.n1 == A && it.n == B) {                                                             \
    plane_run<A, B, A * B / kBatchThreads>(it.src, it.dst, it.tw, it.twp, it.a, plane, lds, \
                                           tid);                                            \
    return;                                                                                  \
  }
  DFT3D_PLANE_CASE(32, 32)
  DFT3D_PLANE_CASE(32, 64)
  DFT3D_PLANE_CASE(32, 128)
  DFT3D_PLANE_CASE(64, 32)
  DFT3D_PLANE_CASE(64, 64)
  DFT3D_PLANE_CASE(128, 32)
#undef DFT3D_PLANE_CASE
}

// A 1D item tile of the persistent kernel, kept out of line so that the
// kernel's registers are those of the largest tile kind, not of all of them
// at once.
template <int N>
__device__ __noinline__ void batch_tile_call(const BatchItem& it, int64_t tile, float2* lds) {
  batch_tile_modes<N>(it, tile, lds);
}

// Wave-uniform copies (lane 0's value) of values every lane holds alike.
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform_i64(long long v) {
  const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)(v & 0xffffffffll));
  const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// All levels of a batch in one launch (see the top of this file).  items
// [0, nitems) in level-major order, total = tickets = sum of ntiles; an
// item's dep is the item of the same problem one level earlier (-1 at level
// 0).  At most spin_limit polls per wait.
//
// Control flow inside the ticket loop is wave-uniform only: the work of
// "thread 0" is done by the whole first wave (branch on the wave index,
// atomics whose operand is 1 on thread 0 and 0 elsewhere) and every wave
// polls for itself.  A divergent `if (threadIdx.x == 0)` block at the end
// of the loop and another at its start were merged by the compiler across
// the back-edge into an inner loop around the barriers from which lane 0
// of the first wave was masked off: the other lanes re-ran the same tile
// forever and the launch never finished.
__global__ void __launch_bounds__(kBatchThreads)
batch_persistent_kernel(const BatchItem* __restrict__ items, int nitems, int64_t total,
                        BatchState* st, unsigned int* done, unsigned int spin_limit) {
  __shared__ float2 lds[kBatchPersistentLds];
  __shared__ long long s_ticket[2];  // [0]: thread 0's ticket; [1]: other lanes' writes
  const int tid = threadIdx.x;
  const unsigned int one = tid == 0 ? 1u : 0u;
  const bool wave0 = uniform_i32(tid) < 64;  // wave-uniform
  for (;;) {
    if (wave0) {
      const unsigned long long t = __hip_atomic_fetch_add(
          &st->head, (unsigned long long)one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_ticket[one ? 0 : 1] = (long long)t;
    }
    __syncthreads();
    const long long ticket = uniform_i64(s_ticket[0]);
    if (ticket >= total) break;
    const int item = uniform_i32(batch_find_item(items, 0, nitems, ticket));
    const BatchItem& it = items[item];
    const int dep = uniform_i32(it.dep);
    if (dep >= 0) {
      // every wave waits for itself (no barrier needed before its loads)
      const unsigned int need = (unsigned int)uniform_i64(items[dep].ntiles);
      unsigned int polls = 0;
      while ((unsigned int)uniform_i32((int)load_relaxed(&done[dep])) < need) {
        ++polls;
        // give up at the limit, or at once when another wait already ran
        // out (the results are then void and reported as such)
        if (polls >= spin_limit ||
            ((polls & 63u) == 0 && uniform_i32((int)load_relaxed(&st->error)) != 0)) {
          __hip_atomic_fetch_or(&st->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      // one acquire per satisfied wait: the producers' stores are visible
      // to this wave's loads from here on
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const int64_t tile = ticket - uniform_i64(it.first);
    if (uniform_i32(it.n1) > 0) {
      batch_small_plane(it, tile, lds, tid);
    } else {
      switch (uniform_i32(it.n)) {
        case 1: batch_tile_call<1>(it, tile, lds); break;
        case 2: batch_tile_call<2>(it, tile, lds); break;
        case 4: batch_tile_call<4>(it, tile, lds); break;
        case 8: batch_tile_call<8>(it, tile, lds); break;
        case 16: batch_tile_call<16>(it, tile, lds); break;
        case 32: batch_tile_call<32>(it, tile, lds); break;
        case 64: batch_tile_call<64>(it, tile, lds); break;
        case 128: batch_tile_call<128>(it, tile, lds); break;
        default: batch_tile_call<256>(it, tile, lds); break;
      }
    }
    // every wave's stores complete and visible device-wide before the tile
    // is counted; the barrier also ends every read of lds and of s_ticket
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave0)
      __hip_atomic_fetch_add(&done[item], one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // The last workgroup to leave zeroes the counters for the next launch:
  // every other workgroup has taken its final ticket by then.
  if (wave0) {
    const unsigned int prev = (unsigned int)uniform_i32((int)__hip_atomic_fetch_add(
        &st->exited, one, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT));
    if (prev + 1 == gridDim.x) {
      for (int i = tid; i < nitems; i += 64)
        __hip_atomic_store(&done[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (tid == 0) {
        __hip_atomic_store(&st->head, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st->exited, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

}  // namespace dft3d
