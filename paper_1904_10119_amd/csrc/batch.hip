// Host side of the batched form (dft3d_execute_batched): turns a sequence
// of plans into the work items of batch_level_kernel (and, for fused plane
// passes, batch_plane_level_kernel) once per sequence of plans; a call
// whose buffers differ from what the device descriptors hold refreshes and
// uploads them, and every call launches one kernel per pass level and item
// kind.  Under stream capture only the launches are recorded.
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/dft3d.h"
#include "batch_kernel.h"
#include "internal.h"

namespace dft3d {

uint64_t next_plan_uid() {
  static std::atomic<uint64_t> counter{1};
  return counter.fetch_add(1);
}

int device_cu_count();

namespace {

int batch_tile_for(int n) {
  switch (n) {
    case 1: return batch_tile<1>();
    case 2: return batch_tile<2>();
    case 4: return batch_tile<4>();
    case 8: return batch_tile<8>();
    case 16: return batch_tile<16>();
    case 32: return batch_tile<32>();
    case 64: return batch_tile<64>();
    case 128: return batch_tile<128>();
    case 256: return batch_tile<256>();
    default: return 0;
  }
}

struct BatchGraph {
  std::vector<const dft3d_plan_s*> plans;
  std::vector<uint64_t> uids;
  std::vector<BatchItem> items;       // host copy (pointers refreshed per call)
  std::vector<int> item_plan, item_pass;
  struct Level {  // one launch: the 1D items or one class of plane items of a pass level
    int item_lo, item_hi;
    int64_t base, ntiles;
    int planes;  // 0: 1D items; 1: small planes; 2: large planes
  };
  std::vector<Level> levels;
  BatchItem* staging = nullptr;       // pinned host copy of the descriptors
  BatchItem* d_items = nullptr;
  // A plan that appears more than once in the batch shares its own
  // workspace with the first occurrence only; later occurrences get one
  // of these (null where the plan's workspace is used).
  std::vector<void*> ws;
  hipEvent_t copied = nullptr;        // the last upload has read staging
  bool launched = false;
  int device = -1;
  // What the device descriptors hold now (per item: source, destination,
  // conjugation flags); a call with the same values needs no upload.
  struct Ptrs {
    const float2* src;
    float2* dst;
    int conj_in, conj_out;
    bool operator==(const Ptrs& o) const {
      return src == o.src && dst == o.dst && conj_in == o.conj_in && conj_out == o.conj_out;
    }
  };
  std::vector<Ptrs> last;
  // Captured into a HIP graph: the descriptors must not change while the
  // plans live; calls with other buffers use another descriptor set.
  bool frozen = false;

  void release() {
    if (copied) {
      (void)hipEventSynchronize(copied);
      (void)hipEventDestroy(copied);
    }
    if (d_items) (void)hipFree(d_items);
    if (staging) (void)hipHostFree(staging);
    for (void* w : ws)
      if (w) (void)hipFree(w);
    ws.clear();
    copied = nullptr;
    d_items = nullptr;
    staging = nullptr;
  }
};

std::mutex g_mutex;
std::vector<BatchGraph*> g_cache;  // most recent last
constexpr size_t kCacheMax = 8;

bool batchable(const dft3d_plan_s* p) {
  for (const Pass& ps : p->passes) {
    if (ps.k->bluestein || ps.k->mixed) return false;
    if (ps.k->plane_rows) {
      if (!batch_plane_shape(ps.k->plane_rows, ps.k->n)) return false;
      continue;
    }
    if (ps.k->n > kBatchMaxN || ps.k->post_twiddle) return false;
    if (batch_tile_for(ps.k->n) == 0) return false;
  }
  return true;
}

// Builds the items (level-major) and the device descriptor buffer.
int build_batch(BatchGraph* g, dft3d_plan_s* const* plans, int count) {
  g->plans.assign(plans, plans + count);
  for (int i = 0; i < count; ++i) g->uids.push_back(plans[i]->uid);
  size_t levels = 0;
  for (int i = 0; i < count; ++i) levels = std::max(levels, plans[i]->passes.size());
  int64_t first = 0;
  for (size_t lv = 0; lv < levels; ++lv) {
    for (int planes = 2; planes >= 0; --planes) {  // large, small planes, then 1D items
      BatchGraph::Level L;
      L.item_lo = (int)g->items.size();
      L.base = first;
      L.planes = planes;
      for (int i = 0; i < count; ++i) {
        const dft3d_plan_s* p = plans[i];
        if (lv >= p->passes.size()) continue;
        const Pass& ps = p->passes[lv];
        const int64_t pts = (int64_t)ps.k->plane_rows * ps.k->n;
        const int kind = ps.k->plane_rows == 0 ? 0 : (pts <= kBatchSmallPlane ? 1 : 2);
        if (kind != planes) continue;
        BatchItem it;
        std::memset(&it, 0, sizeof it);
        it.a = ps.args;
        it.tw = p->tables + p->tw_off[lv];
        it.twp = p->tables + p->twp_off[lv];
        it.n = ps.k->n;
        it.n1 = ps.k->plane_rows;
        it.lmode = ps.k->lmode;
        it.smode = ps.k->smode;
        if (planes) {
          it.ntiles = ps.args.B;
        } else {
          const int T = batch_tile_for(it.n);
          it.ntiles = (ps.args.B + T - 1) / T;
        }
        it.first = first;
        it.dep = -1;
        first += it.ntiles;
        g->items.push_back(it);
        g->item_plan.push_back(i);
        g->item_pass.push_back((int)lv);
      }
      L.item_hi = (int)g->items.size();
      L.ntiles = first - L.base;
      if (L.ntiles > 0x7fffffffLL) return DFT3D_ERR_UNSUPPORTED_SIZE;
      if (L.item_hi > L.item_lo) g->levels.push_back(L);
    }
  }
  g->ws.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    bool repeated = false;
    for (int j = 0; j < i && !repeated; ++j) repeated = plans[j] == plans[i];
    if (repeated && plans[i]->ws_need > 0 &&
        hipMalloc(&g->ws[i], plans[i]->ws_need) != hipSuccess) {
      (void)hipGetLastError();
      return DFT3D_ERR_OUT_OF_MEMORY;
    }
  }
  const size_t bytes = sizeof(BatchItem) * g->items.size();
  if (hipGetDevice(&g->device) != hipSuccess) return DFT3D_ERR_HIP;
  if (hipHostMalloc(reinterpret_cast<void**>(&g->staging), bytes, hipHostMallocDefault) !=
          hipSuccess ||
      hipMalloc(&g->d_items, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return DFT3D_ERR_OUT_OF_MEMORY;
  }
  std::memcpy(g->staging, g->items.data(), bytes);
  if (hipEventCreateWithFlags(&g->copied, hipEventDisableTiming) != hipSuccess)
    return DFT3D_ERR_HIP;
  return DFT3D_OK;
}

// Per-item pointers and flags of a call.
void item_ptrs(const BatchGraph* g, dft3d_plan_s* const* plans, const void* const* in,
               void* const* out, int sign, std::vector<BatchGraph::Ptrs>& cur) {
  cur.resize(g->items.size());
  for (size_t k = 0; k < g->items.size(); ++k) {
    const dft3d_plan_s* p = plans[g->item_plan[k]];
    const Pass& ps = p->passes[g->item_pass[k]];
    const int i = g->item_plan[k];
    void* ws = g->ws[i] ? g->ws[i] : p->ws;
    float2* bufs[3] = {const_cast<float2*>(static_cast<const float2*>(in[i])),
                       static_cast<float2*>(out[i]), static_cast<float2*>(ws)};
    cur[k].src = bufs[ps.src] + ps.in_off;
    cur[k].dst = bufs[ps.dst] + ps.out_off;
    cur[k].conj_in = (sign == 1 && ps.src == BUF_IN) ? 1 : 0;
    cur[k].conj_out = (sign == 1 && g->item_pass[k] + 1 == (int)p->passes.size()) ? 1 : 0;
  }
}

// The cached descriptor set for this sequence of plans: one whose device
// descriptors already match the call if there is one, otherwise one that
// is not frozen (its descriptors get refreshed); null if neither exists.
BatchGraph* find_cached(dft3d_plan_s* const* plans, const void* const* in, void* const* out,
                        int count, int sign, int device, std::vector<BatchGraph::Ptrs>& cur) {
  BatchGraph* reuse = nullptr;
  size_t reuse_at = 0;
  for (size_t c = 0; c < g_cache.size(); ++c) {
    BatchGraph* g = g_cache[c];
    if ((int)g->plans.size() != count || g->device != device) continue;
    bool same = true;
    for (int i = 0; i < count && same; ++i)
      same = g->plans[i] == plans[i] && g->uids[i] == plans[i]->uid;
    if (!same) continue;
    item_ptrs(g, plans, in, out, sign, cur);
    if (g->launched && g->last == cur) {  // move to most recent
      g_cache.erase(g_cache.begin() + (long)c);
      g_cache.push_back(g);
      return g;
    }
    if (!g->frozen && !reuse) {
      reuse = g;
      reuse_at = c;
    }
  }
  if (reuse) {
    g_cache.erase(g_cache.begin() + (long)reuse_at);
    g_cache.push_back(reuse);
    item_ptrs(reuse, plans, in, out, sign, cur);
  }
  return reuse;
}

}  // namespace

int batch_execute(dft3d_plan_s* const* given, const void* const* in, void* const* out,
                  int count, int sign, hipStream_t stream) {
  // Under stream capture only kernel launches may be recorded: the call
  // must find descriptors already on the device for exactly these plans,
  // buffers and sign (left there by an earlier call outside the capture).
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return DFT3D_ERR_HIP;
  }
  if (cs == hipStreamCaptureStatusInvalidated) return DFT3D_ERR_HIP;
  const bool capturing = cs == hipStreamCaptureStatusActive;
  // plans with fused plane passes run as their twins without them
  std::vector<dft3d_plan_s*> views((size_t)count);
  for (int i = 0; i < count; ++i) {
    views[i] = batch_view(given[i]);
    if (!views[i]) return DFT3D_ERR_OUT_OF_MEMORY;
  }
  dft3d_plan_s* const* plans = views.data();
  bool all = true;
  for (int i = 0; i < count; ++i) {
    // a capture cannot allocate: workspaces must exist already
    if (capturing && plans[i]->ws_need > 0 && (!plans[i]->ws || plans[i]->ws_bytes < plans[i]->ws_need))
      return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    const int st = ensure_workspace(plans[i]);
    if (st != DFT3D_OK) return st;
    all = all && batchable(plans[i]);
  }
  if (!all) {  // some pass is too long for the batched kernel: run plan by plan
    for (int i = 0; i < count; ++i) {
      const int st = dft3d_execute(plans[i], in[i], out[i], sign, stream);
      if (st != DFT3D_OK) return st;
    }
    return DFT3D_OK;
  }
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) return DFT3D_ERR_HIP;

  std::lock_guard<std::mutex> lock(g_mutex);
  std::vector<BatchGraph::Ptrs> cur;
  BatchGraph* g = find_cached(plans, in, out, count, sign, device, cur);
  const bool ready = g && g->launched && g->last == cur;
  if (capturing) {
    if (!ready) return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    g->frozen = true;
  } else if (!ready) {
    if (!g) {
      g = new BatchGraph();
      const int st = build_batch(g, plans, count);
      if (st != DFT3D_OK) {
        g->release();
        delete g;
        return st;
      }
      g_cache.push_back(g);
      item_ptrs(g, plans, in, out, sign, cur);
      // evict the oldest set that no graph holds
      if (g_cache.size() > kCacheMax) {
        for (size_t c = 0; c + 1 < g_cache.size(); ++c) {
          if (g_cache[c]->frozen) continue;
          g_cache[c]->release();
          delete g_cache[c];
          g_cache.erase(g_cache.begin() + (long)c);
          break;
        }
      }
    }
    // the previous upload must have read the staging copy before it changes
    if (g->launched && hipEventSynchronize(g->copied) != hipSuccess) return DFT3D_ERR_HIP;
    for (size_t k = 0; k < g->items.size(); ++k) {
      BatchItem& it = g->staging[k];
      it.src = cur[k].src;
      it.dst = cur[k].dst;
      it.a.conj_in = cur[k].conj_in;
      it.a.conj_out = cur[k].conj_out;
    }
    const size_t bytes = sizeof(BatchItem) * g->items.size();
    if (hipMemcpyAsync(g->d_items, g->staging, bytes, hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipEventRecord(g->copied, stream) != hipSuccess)
      return DFT3D_ERR_HIP;
    g->launched = true;
    g->last = cur;
  }
  for (const BatchGraph::Level& L : g->levels) {
    if (L.ntiles <= 0) continue;
    if (L.planes == 1)
      hipLaunchKernelGGL(batch_plane_level_kernel<0>, dim3((unsigned)L.ntiles),
                         dim3(batch_plane_threads<0>()), 0, stream, g->d_items, L.item_lo,
                         L.item_hi, L.base);
    else if (L.planes == 2)
      hipLaunchKernelGGL(batch_plane_level_kernel<1>, dim3((unsigned)L.ntiles),
                         dim3(batch_plane_threads<1>()), 0, stream, g->d_items, L.item_lo,
                         L.item_hi, L.base);
    else
      hipLaunchKernelGGL(batch_level_kernel, dim3((unsigned)L.ntiles), dim3(kBatchThreads), 0,
                         stream, g->d_items, L.item_lo, L.item_hi, L.base);
    if (hipGetLastError() != hipSuccess) return DFT3D_ERR_HIP;
  }
  return DFT3D_OK;
}

bool batch_runs_plane(int n1, int n2) { return batch_plane_shape(n1, n2); }

void batch_forget_plan(const dft3d_plan_s* p) {
  std::lock_guard<std::mutex> lock(g_mutex);
  for (size_t c = 0; c < g_cache.size();) {
    BatchGraph* g = g_cache[c];
    bool uses = false;
    for (const dft3d_plan_s* q : g->plans) uses = uses || q == p;
    if (uses) {
      g->release();
      delete g;
      g_cache.erase(g_cache.begin() + (long)c);
    } else {
      ++c;
    }
  }
}

}  // namespace dft3d
