// Host side of the batched form (dft3d_execute_batched): turns a sequence
// of plans into work items once per sequence of plans; a call whose buffers
// differ from what the device descriptors hold refreshes and uploads them.
//
// Level launches (default): one kernel per pass level and item kind.
// One persistent launch (DFT3D_OPT_BATCH_LAUNCH = 1 on every plan of the
// batch): batch_persistent_kernel runs every level, replayed from a HIP
// graph the library builds once per descriptor set (descriptor upload node,
// then the kernel node; a second graph holds the kernel node alone for calls
// whose descriptors are already on the device).
//
// Under stream capture by the caller only kernel launches are recorded.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <sstream>
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

// One launch of the level form: the 1D items or one class of plane items of
// a pass level.
struct Level {
  int item_lo, item_hi;
  int64_t base, ntiles;
  int planes;  // 0: 1D items; 1: small planes; 2: large planes
};

// Whether every pass of a plan can be a batched item (else the batch runs
// plan by plan).
bool batchable(const std::vector<Pass>& passes, bool persistent) {
  for (const Pass& ps : passes) {
    if (ps.k->bluestein || ps.k->mixed || ps.k->rader || ps.k->halves || ps.k->precision)
      return false;
    if (ps.k->plane_rows) {
      if (!batch_runs_plane(ps.k->plane_rows, ps.k->n, persistent)) return false;
      continue;
    }
    if (ps.k->n > kBatchMaxN || ps.k->post_twiddle) return false;
    if (batch_tile_for(ps.k->n) == 0) return false;
  }
  return true;
}

// Lays the passes of a batch out as items, level-major: for each pass level
// the large planes, the small planes, then the 1D items, problems in order.
// first / ntiles / dep / n / n1 / modes / args are filled, buffer and table
// pointers are left null.  Item k belongs to problem item_plan[k], pass
// item_pass[k]; its dep is the item of the same problem one level earlier.
int batch_layout(const std::vector<const std::vector<Pass>*>& lists, std::vector<BatchItem>& items,
                 std::vector<int>& item_plan, std::vector<int>& item_pass,
                 std::vector<Level>& levels) {
  const int count = (int)lists.size();
  size_t nlev = 0;
  for (const auto* l : lists) nlev = std::max(nlev, l->size());
  std::vector<int> last(count, -1);  // latest item of each problem
  int64_t first = 0;
  for (size_t lv = 0; lv < nlev; ++lv) {
    for (int planes = 2; planes >= 0; --planes) {
      Level L;
      L.item_lo = (int)items.size();
      L.base = first;
      L.planes = planes;
      for (int i = 0; i < count; ++i) {
        if (lv >= lists[i]->size()) continue;
        const Pass& ps = (*lists[i])[lv];
        const int64_t pts = (int64_t)ps.k->plane_rows * ps.k->n;
        const int kind = ps.k->plane_rows == 0 ? 0 : (pts <= kBatchSmallPlane ? 1 : 2);
        if (kind != planes) continue;
        BatchItem it;
        std::memset(&it, 0, sizeof it);
        it.a = ps.args;
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
        it.dep = last[i];
        first += it.ntiles;
        last[i] = (int)items.size();
        items.push_back(it);
        item_plan.push_back(i);
        item_pass.push_back((int)lv);
      }
      L.item_hi = (int)items.size();
      L.ntiles = first - L.base;
      if (L.ntiles > 0x7fffffffLL || first > 0x7fffffffLL) return DFT3D_ERR_UNSUPPORTED_SIZE;
      if (L.item_hi > L.item_lo) levels.push_back(L);
    }
  }
  return DFT3D_OK;
}

// Poll limit of one dependency wait in the persistent kernel (each poll is
// a device-scope load and a short sleep, about a microsecond): 2^20 polls
// is about a second, far above any real wait.  DFT3D_BATCH_SPIN_LIMIT
// overrides it (tests force the limit to be reached).
unsigned int spin_limit() {
  const char* e = std::getenv("DFT3D_BATCH_SPIN_LIMIT");
  if (e && *e) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= 0x7fffffffL) return (unsigned int)v;
  }
  return 1u << 20;
}

// DFT3D_BATCH_CHECK=1: persistent calls wait for the launch to finish and
// return DFT3D_ERR_HIP if a dependency wait ran out (the flag is cleared).
bool batch_check() {
  const char* e = std::getenv("DFT3D_BATCH_CHECK");
  return e && std::strcmp(e, "1") == 0;
}

struct BatchGraph {
  std::vector<const dft3d_plan_s*> plans;
  std::vector<uint64_t> uids;
  bool persistent = false;
  std::vector<BatchItem> items;       // host copy (pointers refreshed per call)
  std::vector<int> item_plan, item_pass;
  std::vector<Level> levels;
  BatchItem* staging = nullptr;       // pinned host copy of the descriptors
  BatchItem* d_items = nullptr;
  // Workspaces of problems that cannot use their plan's own: a plan that
  // appears more than once, or whose bound workspace overlaps the workspace
  // of an earlier problem of the batch (null where the plan's is used).
  std::vector<void*> ws;
  hipEvent_t copied = nullptr;        // the last upload has read staging
  bool launched = false;
  int device = -1;
  // Persistent form: counters, grid, and the two graphs (upload + kernel,
  // kernel alone).
  BatchState* d_state = nullptr;
  unsigned int* d_done = nullptr;
  int64_t total = 0;
  unsigned int grid = 0;
  unsigned int spin = 0;
  hipGraph_t graph_full = nullptr, graph_kernel = nullptr;
  hipGraphExec_t exec_full = nullptr, exec_kernel = nullptr;
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
    if (exec_full) (void)hipGraphExecDestroy(exec_full);
    if (exec_kernel) (void)hipGraphExecDestroy(exec_kernel);
    if (graph_full) (void)hipGraphDestroy(graph_full);
    if (graph_kernel) (void)hipGraphDestroy(graph_kernel);
    if (d_items) (void)hipFree(d_items);
    if (d_state) (void)hipFree(d_state);
    if (d_done) (void)hipFree(d_done);
    if (staging) (void)hipHostFree(staging);
    for (void* w : ws)
      if (w) (void)hipFree(w);
    ws.clear();
    copied = nullptr;
    exec_full = exec_kernel = nullptr;
    graph_full = graph_kernel = nullptr;
    d_items = nullptr;
    d_state = nullptr;
    d_done = nullptr;
    staging = nullptr;
  }
};

std::mutex g_mutex;
std::vector<BatchGraph*> g_cache;  // most recent last
constexpr size_t kCacheMax = 8;

// Problems that need a private workspace: a repeated plan, or a plan whose
// workspace overlaps the one an earlier problem of the batch uses (distinct
// plans may be bound to one caller buffer for dft3d_execute, where calls are
// ordered; in one batched call their passes run at the same time).
std::vector<bool> private_ws_needed(dft3d_plan_s* const* plans, int count) {
  std::vector<bool> need((size_t)count, false);
  for (int i = 0; i < count; ++i) {
    const dft3d_plan_s* p = plans[i];
    if (p->ws_need == 0) continue;
    for (int j = 0; j < i && !need[i]; ++j) {
      const dft3d_plan_s* q = plans[j];
      if (q == p) {
        need[i] = true;
      } else if (q->ws_need > 0 && !need[j]) {
        const char* a = static_cast<const char*>(p->ws);
        const char* b = static_cast<const char*>(q->ws);
        need[i] = a < b + q->ws_need && b < a + p->ws_need;
      }
    }
  }
  return need;
}

// Grid of the persistent kernel: resident workgroups, at most one per ticket.
int persistent_grid(int64_t total, unsigned int& grid) {
  static int per_cu = -1;
  if (per_cu < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_persistent_kernel, kBatchThreads,
                                                     0) != hipSuccess) {
      (void)hipGetLastError();
      return DFT3D_ERR_HIP;
    }
    per_cu = nb > 0 ? nb : 1;
  }
  int64_t g = (int64_t)device_cu_count() * per_cu;
  if (g > total) g = total;
  grid = (unsigned int)(g > 0 ? g : 1);
  return DFT3D_OK;
}

// The two graphs of the persistent form.
int build_graphs(BatchGraph* g) {
  const size_t bytes = sizeof(BatchItem) * g->items.size();
  int nitems = (int)g->items.size();
  void* args[] = {&g->d_items, &nitems, &g->total, &g->d_state, &g->d_done, &g->spin};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof kp);
  kp.func = reinterpret_cast<void*>(batch_persistent_kernel);
  kp.gridDim = dim3(g->grid);
  kp.blockDim = dim3(kBatchThreads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  hipGraphNode_t copy = nullptr, kern = nullptr, kern2 = nullptr;
  if (hipGraphCreate(&g->graph_full, 0) != hipSuccess ||
      hipGraphAddMemcpyNode1D(&copy, g->graph_full, nullptr, 0, g->d_items, g->staging, bytes,
                              hipMemcpyHostToDevice) != hipSuccess ||
      hipGraphAddKernelNode(&kern, g->graph_full, &copy, 1, &kp) != hipSuccess ||
      hipGraphInstantiate(&g->exec_full, g->graph_full, nullptr, nullptr, 0) != hipSuccess ||
      hipGraphCreate(&g->graph_kernel, 0) != hipSuccess ||
      hipGraphAddKernelNode(&kern2, g->graph_kernel, nullptr, 0, &kp) != hipSuccess ||
      hipGraphInstantiate(&g->exec_kernel, g->graph_kernel, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    return DFT3D_ERR_HIP;
  }
  return DFT3D_OK;
}

// Builds the items and the device descriptor buffer (and, for the
// persistent form, its counters and graphs).
int build_batch(BatchGraph* g, dft3d_plan_s* const* plans, int count, bool persistent,
                hipStream_t stream) {
  g->plans.assign(plans, plans + count);
  for (int i = 0; i < count; ++i) g->uids.push_back(plans[i]->uid);
  g->persistent = persistent;
  std::vector<const std::vector<Pass>*> lists;
  for (int i = 0; i < count; ++i) lists.push_back(&plans[i]->passes);
  int st = batch_layout(lists, g->items, g->item_plan, g->item_pass, g->levels);
  if (st != DFT3D_OK) return st;
  for (size_t k = 0; k < g->items.size(); ++k) {
    const dft3d_plan_s* p = plans[g->item_plan[k]];
    const int lv = g->item_pass[k];
    g->items[k].tw = p->tables + p->tw_off[lv];
    g->items[k].twp = p->tables + p->twp_off[lv];
  }
  g->ws.assign(count, nullptr);
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
  if (persistent) {
    g->total = 0;
    for (const BatchItem& it : g->items) g->total += it.ntiles;
    g->spin = spin_limit();
    if (hipMalloc(&g->d_state, sizeof(BatchState)) != hipSuccess ||
        hipMalloc(&g->d_done, sizeof(unsigned int) * g->items.size()) != hipSuccess) {
      (void)hipGetLastError();
      return DFT3D_ERR_OUT_OF_MEMORY;
    }
    // the counters start at zero (in stream order before the first launch;
    // never under capture); every launch leaves them at zero
    if (hipMemsetAsync(g->d_state, 0, sizeof(BatchState), stream) != hipSuccess ||
        hipMemsetAsync(g->d_done, 0, sizeof(unsigned int) * g->items.size(), stream) !=
            hipSuccess) {
      (void)hipGetLastError();
      return DFT3D_ERR_HIP;
    }
    st = persistent_grid(g->total, g->grid);
    if (st != DFT3D_OK) return st;
    st = build_graphs(g);
    if (st != DFT3D_OK) return st;
  }
  return DFT3D_OK;
}

// Private workspaces the call needs that the descriptor set does not have
// yet; not allowed under capture.
int ensure_private_ws(BatchGraph* g, dft3d_plan_s* const* plans, int count, bool capturing) {
  const std::vector<bool> need = private_ws_needed(plans, count);
  for (int i = 0; i < count; ++i) {
    if (!need[i] || g->ws[i]) continue;
    if (capturing) return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    if (hipMalloc(&g->ws[i], plans[i]->ws_need) != hipSuccess) {
      (void)hipGetLastError();
      g->ws[i] = nullptr;
      return DFT3D_ERR_OUT_OF_MEMORY;
    }
  }
  return DFT3D_OK;
}

// Per-item pointers and flags of a call.
void item_ptrs(const BatchGraph* g, dft3d_plan_s* const* plans, const void* const* in,
               void* const* out, int sign, std::vector<BatchGraph::Ptrs>& cur) {
  cur.resize(g->items.size());
  const std::vector<bool> need = private_ws_needed(plans, (int)g->plans.size());
  for (size_t k = 0; k < g->items.size(); ++k) {
    const dft3d_plan_s* p = plans[g->item_plan[k]];
    const Pass& ps = p->passes[g->item_pass[k]];
    const int i = g->item_plan[k];
    void* ws = need[i] ? g->ws[i] : p->ws;
    float2* bufs[3] = {const_cast<float2*>(static_cast<const float2*>(in[i])),
                       static_cast<float2*>(out[i]), static_cast<float2*>(ws)};
    cur[k].src = bufs[ps.src] + ps.in_off;
    cur[k].dst = bufs[ps.dst] + ps.out_off;
    cur[k].conj_in = (sign == 1 && ps.src == BUF_IN) ? 1 : 0;
    cur[k].conj_out = (sign == 1 && g->item_pass[k] + 1 == (int)p->passes.size()) ? 1 : 0;
  }
}

// The cached descriptor set for this sequence of plans and form: one whose
// device descriptors already match the call if there is one, otherwise one
// that is not frozen (its descriptors get refreshed); null if neither exists.
BatchGraph* find_cached(dft3d_plan_s* const* plans, const void* const* in, void* const* out,
                        int count, int sign, int device, bool persistent,
                        std::vector<BatchGraph::Ptrs>& cur) {
  BatchGraph* reuse = nullptr;
  size_t reuse_at = 0;
  for (size_t c = 0; c < g_cache.size(); ++c) {
    BatchGraph* g = g_cache[c];
    if ((int)g->plans.size() != count || g->device != device || g->persistent != persistent)
      continue;
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
  }
  return reuse;
}

// Launches of the level form.
int launch_levels(const BatchGraph* g, hipStream_t stream) {
  for (const Level& L : g->levels) {
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

// After a persistent launch in check mode: wait for it, read and clear the
// error flag.
int check_persistent(BatchGraph* g, hipStream_t stream) {
  if (hipStreamSynchronize(stream) != hipSuccess) return DFT3D_ERR_HIP;
  unsigned int err = 0;
  if (hipMemcpy(&err, &g->d_state->error, sizeof err, hipMemcpyDeviceToHost) != hipSuccess)
    return DFT3D_ERR_HIP;
  if (err) {
    const unsigned int zero = 0;
    if (hipMemcpy(&g->d_state->error, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
      return DFT3D_ERR_HIP;
    return DFT3D_ERR_HIP;
  }
  return DFT3D_OK;
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
  // the one-launch form when every plan asks for it
  bool persistent = count > 0;
  for (int i = 0; i < count; ++i) persistent = persistent && given[i]->opt.batch_launch == 1;
  // plans with fused plane passes the form does not cover run as their
  // twins without them
  std::vector<dft3d_plan_s*> views((size_t)count);
  for (int i = 0; i < count; ++i) {
    views[i] = batch_view(given[i], persistent);
    if (!views[i]) return DFT3D_ERR_OUT_OF_MEMORY;
  }
  dft3d_plan_s* const* plans = views.data();
  bool all = true;
  for (int i = 0; i < count; ++i) {
    // a capture cannot allocate: workspaces must exist already
    if (capturing && plans[i]->ws_need > 0 &&
        (!plans[i]->ws || plans[i]->ws_bytes < plans[i]->ws_need))
      return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    const int st = ensure_workspace(plans[i]);
    if (st != DFT3D_OK) return st;
    all = all && batchable(plans[i]->passes, persistent);
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
  BatchGraph* g = find_cached(plans, in, out, count, sign, device, persistent, cur);
  if (!g && !capturing) {
    g = new BatchGraph();
    const int st = build_batch(g, plans, count, persistent, stream);
    if (st != DFT3D_OK) {
      g->release();
      delete g;
      return st;
    }
    g_cache.push_back(g);
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
  if (!g) return DFT3D_ERR_UNSUPPORTED_SCHEDULE;  // capturing without descriptors
  {
    const int st = ensure_private_ws(g, plans, count, capturing);
    if (st != DFT3D_OK) return st;
  }
  item_ptrs(g, plans, in, out, sign, cur);
  const bool ready = g->launched && g->last == cur;
  if (capturing) {
    if (!ready) return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    g->frozen = true;
    if (!g->persistent) return launch_levels(g, stream);
    hipLaunchKernelGGL(batch_persistent_kernel, dim3(g->grid), dim3(kBatchThreads), 0, stream,
                       g->d_items, (int)g->items.size(), g->total, g->d_state, g->d_done,
                       g->spin);
    return hipGetLastError() == hipSuccess ? DFT3D_OK : DFT3D_ERR_HIP;
  }
  if (!ready) {
    // the previous upload must have read the staging copy before it changes
    if (g->launched && hipEventSynchronize(g->copied) != hipSuccess) return DFT3D_ERR_HIP;
    for (size_t k = 0; k < g->items.size(); ++k) {
      BatchItem& it = g->staging[k];
      it.src = cur[k].src;
      it.dst = cur[k].dst;
      it.a.conj_in = cur[k].conj_in;
      it.a.conj_out = cur[k].conj_out;
    }
  }
  if (!g->persistent) {
    if (!ready) {
      const size_t bytes = sizeof(BatchItem) * g->items.size();
      if (hipMemcpyAsync(g->d_items, g->staging, bytes, hipMemcpyHostToDevice, stream) !=
              hipSuccess ||
          hipEventRecord(g->copied, stream) != hipSuccess)
        return DFT3D_ERR_HIP;
      g->launched = true;
      g->last = cur;
    }
    return launch_levels(g, stream);
  }
  // persistent: replay the upload + kernel graph, or the kernel alone; the
  // event marks the end of the launch (staging read, counters free again)
  if (hipGraphLaunch(ready ? g->exec_kernel : g->exec_full, stream) != hipSuccess ||
      hipEventRecord(g->copied, stream) != hipSuccess) {
    (void)hipGetLastError();
    return DFT3D_ERR_HIP;
  }
  g->launched = true;
  g->last = cur;
  return batch_check() ? check_persistent(g, stream) : DFT3D_OK;
}

bool batch_runs_plane(int n1, int n2, bool persistent) {
  return persistent ? batch_persistent_plane_shape(n1, n2) : batch_plane_shape(n1, n2);
}

std::string batch_describe(const std::vector<const std::vector<Pass>*>& lists,
                           bool persistent) {
  std::ostringstream os;
  bool all = true;
  for (const auto* l : lists) all = all && batchable(*l, persistent);
  os << "{\"launch\":\"" << (persistent ? "persistent" : "levels") << "\",\"batchable\":"
     << (all ? "true" : "false") << ",\"threads\":" << kBatchThreads;
  if (persistent)
    os << ",\"lds_bytes\":" << (int)(sizeof(float2) * kBatchPersistentLds);
  std::vector<BatchItem> items;
  std::vector<int> item_plan, item_pass;
  std::vector<Level> levels;
  int64_t total = 0;
  if (all && batch_layout(lists, items, item_plan, item_pass, levels) != DFT3D_OK) all = false;
  for (const BatchItem& it : items) total += it.ntiles;
  os << ",\"total\":" << total << ",\"items\":[";
  for (size_t k = 0; k < items.size(); ++k) {
    const BatchItem& it = items[k];
    os << (k ? "," : "") << "{\"problem\":" << item_plan[k] << ",\"pass\":" << item_pass[k]
       << ",\"first\":" << it.first << ",\"ntiles\":" << it.ntiles << ",\"dep\":" << it.dep
       << ",\"n\":" << it.n << ",\"n1\":" << it.n1 << ",\"pencils\":" << it.a.B
       << ",\"tile\":" << (it.n1 ? 1 : batch_tile_for(it.n)) << "}";
  }
  os << "],\"levels\":[";
  for (size_t k = 0; k < levels.size(); ++k) {
    const Level& L = levels[k];
    os << (k ? "," : "") << "{\"item_lo\":" << L.item_lo << ",\"item_hi\":" << L.item_hi
       << ",\"base\":" << L.base << ",\"ntiles\":" << L.ntiles << ",\"planes\":" << L.planes
       << "}";
  }
  os << "]}";
  return os.str();
}

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
