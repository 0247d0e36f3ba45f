// C ABI of libdft3d.so (declared in include/dft3d.h): plan life cycle, table
// upload, workspace management and pass launches.
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>

#include "../../include/dft3d.h"
#include "internal.h"

using namespace dft3d;

namespace {

// Test hook: DFT3D_FAULT_INJECT=alloc|upload|launch forces that step to
// fail so the error paths can be exercised.
bool fault(const char* what) {
  const char* e = std::getenv("DFT3D_FAULT_INJECT");
  return e && std::strcmp(e, what) == 0;
}

// DFT3D_MAX_WORKSPACE_BYTES: plan-owned workspaces above this many bytes are
// refused with DFT3D_ERR_OUT_OF_MEMORY instead of being allocated (a cap for
// shared devices; also forces the out-of-memory path in tests).
bool workspace_over_cap(size_t bytes) {
  const char* e = std::getenv("DFT3D_MAX_WORKSPACE_BYTES");
  if (!e || !*e) return false;
  char* end = nullptr;
  const unsigned long long cap = std::strtoull(e, &end, 10);
  return end && *end == '\0' && bytes > cap;
}

int validate(int64_t n0, int64_t n1, int64_t n2, int schedule, int layout) {
  if (schedule < DFT3D_SCHED_AUTO || schedule > DFT3D_SCHED_VOLUMETRIC)
    return DFT3D_ERR_INVALID_ARG;
  if (layout != DFT3D_LAYOUT_NATURAL && layout != DFT3D_LAYOUT_SHUFFLED)
    return DFT3D_ERR_INVALID_ARG;
  const int64_t n[3] = {n0, n1, n2};
  for (int d = 0; d < 3; ++d) {
    if (!length_supported(n[d])) return DFT3D_ERR_UNSUPPORTED_SIZE;
  }
  return DFT3D_OK;
}

void free_tables(dft3d_plan_s* p) {
  if (p->tables) (void)hipFree(p->tables);
  p->tables = nullptr;
}

void free_workspace(dft3d_plan_s* p) {
  if (p->ws_owned && p->ws) (void)hipFree(p->ws);
  if (p->ws_owned) {
    p->ws = nullptr;
    p->ws_bytes = 0;
  }
  p->ws_owned = false;
}

// (Re)build the pass list and upload one root table per distinct length.
int rebuild(dft3d_plan_s* p) {
  std::vector<Pass> passes;
  size_t ws = 0;
  int resolved = 0;
  const int sched = (p->schedule == DFT3D_SCHED_AUTO && p->tuned >= 0) ? p->tuned : p->schedule;
  int st = build_passes(p->n, sched, p->layout, p->opt, passes, ws, resolved);
  if (st != DFT3D_OK) return st;
  // shuffled plans: the inverse runs its own list (shuffled in, natural out)
  std::vector<Pass> ipasses;
  if (p->layout == DFT3D_LAYOUT_SHUFFLED) {
    size_t iws = 0;
    int ires = 0;
    st = build_passes(p->n, sched, p->layout, p->opt, ipasses, iws, ires, true);
    if (st != DFT3D_OK) return st;
    if (iws > ws) ws = iws;
  }

  // one table per distinct root length (key n > 0) and per MFMA leaf
  // precision (key -precision, kLeafTableFloat2 slots of 16-bit values);
  // Bluestein chirp and filter tables per length n (keys (1, n), (2, n),
  // the filter stored right after the chirp)
  std::map<int64_t, int64_t> offsets;
  std::map<std::pair<int, int64_t>, int64_t> bl_offsets;
  // mixed-radix stage twiddles per length n and radix code (value: offset)
  std::map<std::pair<int64_t, uint64_t>, int64_t> mx_offsets;
  // Rader tables per prime length n (value: offset)
  std::map<int64_t, int64_t> rd_offsets;
  int64_t total = 0;
  std::vector<const Pass*> all;
  for (const Pass& ps : passes) all.push_back(&ps);
  for (const Pass& ps : ipasses) all.push_back(&ps);
  // every table-carrying pass has its length (a kernel picked for the wrong
  // kind of pass would size its tables from zero)
  for (const Pass* pp : all)
    if ((pp->k->rader && pp->rader_n < 3) || (pp->k->mixed && pp->args.res_mask < 2) ||
        (pp->k->bluestein && pp->bl_n < 1))
      return DFT3D_ERR_UNSUPPORTED_SIZE;
  for (const Pass* pp : all) {
    const Pass& ps = *pp;
    if (ps.k->rader) {  // stage twiddles of n - 1, and the Rader tables of n
      const std::pair<int64_t, uint64_t> key{ps.rader_n - 1, (uint64_t)ps.args.twp_mask};
      if (!mx_offsets.count(key)) {
        mx_offsets[key] = total;
        total += key.first;
      }
      if (!rd_offsets.count(ps.rader_n)) {
        rd_offsets[ps.rader_n] = total;
        total += rader_table_size(ps.rader_n);
      }
      continue;
    }
    if (ps.k->mixed) {
      const std::pair<int64_t, uint64_t> key{ps.args.res_mask, (uint64_t)ps.args.twp_mask};
      if (!mx_offsets.count(key)) {
        mx_offsets[key] = total;
        total += key.first;
      }
      continue;
    }
    for (int64_t len : {ps.tw_len, ps.twp_len}) {
      if (len > 0 && !offsets.count(len)) {
        offsets[len] = total;
        total += len;
      }
    }
    if (ps.leaf && !offsets.count(-ps.leaf)) {
      offsets[-ps.leaf] = total;
      total += kLeafTableFloat2;
    }
    if (ps.k->bluestein && !bl_offsets.count({1, ps.bl_n})) {
      bl_offsets[{1, ps.bl_n}] = total;
      total += ps.bl_n;
      bl_offsets[{2, ps.bl_n}] = total;
      total += bluestein_length(ps.bl_n);
    }
  }
  std::vector<float2> host((size_t)total);
  for (auto& kv : offsets) {
    if (kv.first > 0)
      make_roots(kv.first, host.data() + kv.second);
    else
      make_leaf_table((int)-kv.first, reinterpret_cast<unsigned short*>(host.data() + kv.second));
  }
  for (auto& kv : mx_offsets)
    make_mixed_twiddles(kv.first.first, kv.first.second, host.data() + kv.second);
  for (auto& kv : rd_offsets) make_rader_tables(kv.first, host.data() + kv.second);
  for (auto& kv : bl_offsets) {
    if (kv.first.first == 1)
      make_chirp(kv.first.second, host.data() + kv.second);
    else
      make_bluestein_filter(kv.first.second, host.data() + kv.second);
  }

  float2* dev = nullptr;
  if (fault("alloc") || hipMalloc(&dev, sizeof(float2) * (size_t)total) != hipSuccess) {
    (void)hipGetLastError();
    return DFT3D_ERR_OUT_OF_MEMORY;
  }
  if (fault("upload") || hipMemcpy(dev, host.data(), sizeof(float2) * (size_t)total,
                                   hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(dev);
    return DFT3D_ERR_HIP;
  }
  free_tables(p);
  p->tables = dev;
  p->passes.swap(passes);
  p->ipasses.swap(ipasses);
  auto table_offsets = [&offsets, &bl_offsets, &mx_offsets, &rd_offsets](
                           const std::vector<Pass>& list, std::vector<int64_t>& tw,
                           std::vector<int64_t>& twp) {
    tw.clear();
    twp.clear();
    for (const Pass& ps : list) {
      if (ps.k->rader) {
        tw.push_back(mx_offsets[{ps.rader_n - 1, (uint64_t)ps.args.twp_mask}]);
        twp.push_back(rd_offsets[ps.rader_n]);
        continue;
      }
      if (ps.k->mixed) {  // the stage twiddles of the length
        tw.push_back(mx_offsets[{ps.args.res_mask, (uint64_t)ps.args.twp_mask}]);
        twp.push_back(0);
        continue;
      }
      if (ps.k->bluestein) {  // roots of m; the chirp, with the filter right after it
        tw.push_back(offsets[ps.tw_len]);
        twp.push_back(bl_offsets[{1, ps.bl_n}]);
        continue;
      }
      tw.push_back(offsets[ps.tw_len]);
      // post-twiddle table, or the leaf operand table for MFMA passes
      twp.push_back(ps.leaf ? offsets[-ps.leaf] : (ps.twp_len > 0 ? offsets[ps.twp_len] : 0));
    }
  };
  table_offsets(p->passes, p->tw_off, p->twp_off);
  table_offsets(p->ipasses, p->itw_off, p->itwp_off);
  p->resolved = resolved;
  p->uid = next_plan_uid();
  if (ws > p->ws_need && p->ws_owned) free_workspace(p);  // regrown lazily
  p->ws_need = ws;
  return DFT3D_OK;
}

bool overlaps(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

// Applies one option to an Options value; returns a status.
int apply_option(Options& o, int key, int64_t value) {
  switch (key) {
    case DFT3D_OPT_PRECISION:
      if (value < DFT3D_PREC_FP32 || value > DFT3D_PREC_FP16X3) return DFT3D_ERR_INVALID_ARG;
      o.precision = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_TILE:
      if (value < 0 || value > 4096 || (value & (value - 1)) != 0) return DFT3D_ERR_INVALID_ARG;
      o.tile = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_XCD_REMAP:
      if (value != 0 && value != 1) return DFT3D_ERR_INVALID_ARG;
      o.xcd_remap = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_SPLIT_MAX:
      if (value < 0 || value > 4096) return DFT3D_ERR_INVALID_ARG;
      o.split_max = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_NONTEMPORAL:
      if (value < 0 || value > 2) return DFT3D_ERR_INVALID_ARG;
      o.nontemporal = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_PERSISTENT:
      if (value != 0 && value != 1) return DFT3D_ERR_INVALID_ARG;
      o.persistent = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_SLAB_GROUP:
      if (value < -1 || value > 4096) return DFT3D_ERR_INVALID_ARG;
      o.slab_group = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_FUSED_PLANE:
      if (value != 0 && value != 1) return DFT3D_ERR_INVALID_ARG;
      o.fused_plane = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_FUSED_AXES:
      if (value != 0 && value != 1) return DFT3D_ERR_INVALID_ARG;
      o.fused_axes = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_PENCIL_GROUP:
      if (value < -1 || value > 4096) return DFT3D_ERR_INVALID_ARG;
      o.pencil_group = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_BATCH_LAUNCH:
      if (value != 0 && value != 1) return DFT3D_ERR_INVALID_ARG;
      o.batch_launch = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_MOVE_ONLY:
      if (value < 0 || value > 2) return DFT3D_ERR_INVALID_ARG;
      o.move_only = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_MFMA_LEAF:
      if (value != 0 && value != 16 && value != 32) return DFT3D_ERR_INVALID_ARG;
      o.mfma_leaf = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_RADICES:
      if (!radix_code_valid((uint64_t)value)) return DFT3D_ERR_INVALID_ARG;
      o.radices = (uint64_t)value;
      return DFT3D_OK;
    case DFT3D_OPT_RADER:
      if (value < 0 || value > 2) return DFT3D_ERR_INVALID_ARG;
      o.rader = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_HALVES:
      if (value < 0 || value > 1) return DFT3D_ERR_INVALID_ARG;
      o.halves = (int)value;
      return DFT3D_OK;
    case DFT3D_OPT_PENCIL_ORDER:
      if (value < -1 || value > 2) return DFT3D_ERR_INVALID_ARG;
      o.pencil_order = (int)value;
      return DFT3D_OK;
    default:
      return DFT3D_ERR_INVALID_ARG;
  }
}

}  // namespace

namespace dft3d {
void destroy_twin(dft3d_plan_s* p) {
  if (!p->batch_twin) return;
  batch_forget_plan(p->batch_twin);
  free_workspace(p->batch_twin);
  free_tables(p->batch_twin);
  delete p->batch_twin;
  p->batch_twin = nullptr;
}

dft3d_plan_s* batch_view(dft3d_plan_s* p, bool persistent) {
  bool plane = false;
  for (const Pass& ps : p->passes)
    plane = plane ||
            (ps.k->plane_rows > 0 && !batch_runs_plane(ps.k->plane_rows, ps.k->n, persistent));
  if (!plane) return p;
  if (p->batch_twin) return p->batch_twin;
  dft3d_plan_s* t = new (std::nothrow) dft3d_plan_s();
  if (!t) return nullptr;
  for (int d = 0; d < 3; ++d) t->n[d] = p->n[d];
  t->schedule = p->schedule;
  t->layout = p->layout;
  t->opt = p->opt;
  t->opt.fused_plane = 0;
  t->device = p->device;
  t->tuned = p->tuned;
  if (rebuild(t) != DFT3D_OK) {
    free_tables(t);
    delete t;
    return nullptr;
  }
  p->batch_twin = t;
  return t;
}

int ensure_workspace(dft3d_plan_s* p) {
  if (p->ws_need > 0 && (!p->ws || p->ws_bytes < p->ws_need)) {
    if (!p->ws_owned && p->ws) return DFT3D_ERR_WORKSPACE_TOO_SMALL;
    free_workspace(p);
    void* w = nullptr;
    if (fault("alloc") || workspace_over_cap(p->ws_need) ||
        hipMalloc(&w, p->ws_need) != hipSuccess) {
      (void)hipGetLastError();
      return DFT3D_ERR_OUT_OF_MEMORY;
    }
    p->ws = w;
    p->ws_bytes = p->ws_need;
    p->ws_owned = true;
  }
  return DFT3D_OK;
}

int check_device(const dft3d_plan_s* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return DFT3D_ERR_HIP;
  }
  return dev == p->device ? DFT3D_OK : DFT3D_ERR_INVALID_ARG;
}

int execute_passes(dft3d_plan_s* p, const void* in, void* out, int sign, hipStream_t s,
                   void* ws) {
  const size_t bytes = (size_t)(p->n[0] * p->n[1] * p->n[2]) * sizeof(float2);
  if (p->ws_need > 0 && (!ws || overlaps(ws, in, bytes) || overlaps(ws, out, bytes)))
    return DFT3D_ERR_INVALID_ARG;
  if (fault("launch")) return DFT3D_ERR_HIP;
  float2* bufs[3] = {const_cast<float2*>(static_cast<const float2*>(in)),
                     static_cast<float2*>(out), static_cast<float2*>(ws)};
  // a shuffled plan's inverse takes shuffled input through its own list
  const bool inv_list = sign == 1 && !p->ipasses.empty();
  const std::vector<Pass>& list = inv_list ? p->ipasses : p->passes;
  const std::vector<int64_t>& tw_off = inv_list ? p->itw_off : p->tw_off;
  const std::vector<int64_t>& twp_off = inv_list ? p->itwp_off : p->twp_off;
  const size_t np = list.size();
  for (size_t i = 0; i < np; ++i) {
    const Pass& ps = list[i];
    PassArgs a = ps.args;
    // inverse as conj(DFT(conj(x))): every pass reading the input conjugates
    // it; the last pass writes every output element and conjugates them
    a.conj_in = (sign == 1 && ps.src == BUF_IN) ? 1 : 0;
    a.conj_out = (sign == 1 && i + 1 == np) ? 1 : 0;
    const float2* tw = p->tables + tw_off[i];
    const float2* twp = p->tables + twp_off[i];
    hipError_t e =
        ps.k->launch(a, bufs[ps.src] + ps.in_off, bufs[ps.dst] + ps.out_off, tw, twp, s);
    if (e != hipSuccess) return DFT3D_ERR_HIP;
  }
  return DFT3D_OK;
}
}  // namespace dft3d

extern "C" {

const char* dft3d_status_string(int status) {
  switch (status) {
    case DFT3D_OK: return "ok";
    case DFT3D_ERR_INVALID_ARG: return "invalid argument";
    case DFT3D_ERR_UNSUPPORTED_SIZE:
      return "unsupported size (each n_d must be in [1, 4096])";
    case DFT3D_ERR_UNSUPPORTED_SCHEDULE: return "unsupported schedule/layout/precision combination";
    case DFT3D_ERR_NO_DEVICE: return "no HIP device";
    case DFT3D_ERR_OUT_OF_MEMORY: return "device out of memory";
    case DFT3D_ERR_HIP: return "HIP runtime error";
    case DFT3D_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    default: return "unknown status";
  }
}

int dft3d_plan_describe(int64_t n0, int64_t n1, int64_t n2, int schedule, int layout,
                        const int* keys, const int64_t* values, int nopts, char* buf,
                        size_t len, size_t* needed) {
  int st = validate(n0, n1, n2, schedule, layout);
  if (st != DFT3D_OK) return st;
  if (nopts < 0 || (nopts > 0 && (!keys || !values))) return DFT3D_ERR_INVALID_ARG;
  Options opt;
  for (int i = 0; i < nopts; ++i) {
    st = apply_option(opt, keys[i], values[i]);
    if (st != DFT3D_OK) return st;
  }
  const int64_t n[3] = {n0, n1, n2};
  std::vector<Pass> passes;
  size_t ws = 0;
  int resolved = 0;
  st = build_passes(n, schedule, layout, opt, passes, ws, resolved);
  if (st != DFT3D_OK) return st;
  std::vector<Pass> ipasses;
  if (layout == DFT3D_LAYOUT_SHUFFLED) {
    size_t iws = 0;
    int ires = 0;
    st = build_passes(n, schedule, layout, opt, ipasses, iws, ires, true);
    if (st != DFT3D_OK) return st;
    if (iws > ws) ws = iws;
  }
  const std::string s = describe_passes(n, resolved, layout, passes,
                                        layout == DFT3D_LAYOUT_SHUFFLED ? &ipasses : nullptr, ws);
  if (needed) *needed = s.size() + 1;
  if (buf && len > 0) {
    const size_t m = s.size() < len - 1 ? s.size() : len - 1;
    std::memcpy(buf, s.data(), m);
    buf[m] = '\0';
  }
  return DFT3D_OK;
}

int dft3d_batch_describe(const int64_t* shapes, int count, int schedule, int launch,
                         char* buf, size_t len, size_t* needed) {
  if (count < 0 || (count > 0 && !shapes) || (launch != 0 && launch != 1))
    return DFT3D_ERR_INVALID_ARG;
  std::vector<std::vector<Pass>> lists((size_t)count);
  for (int i = 0; i < count; ++i) {
    const int64_t* n = shapes + 3 * i;
    int st = validate(n[0], n[1], n[2], schedule, DFT3D_LAYOUT_NATURAL);
    if (st != DFT3D_OK) return st;
    Options opt;
    opt.batch_launch = launch;
    size_t ws = 0;
    int resolved = 0;
    st = build_passes(n, schedule, DFT3D_LAYOUT_NATURAL, opt, lists[i], ws, resolved);
    if (st != DFT3D_OK) return st;
    // as batch_view: plane passes the form does not cover run unfused
    bool uncovered = false;
    for (const Pass& ps : lists[i])
      uncovered = uncovered || (ps.k->plane_rows > 0 &&
                                !batch_runs_plane(ps.k->plane_rows, ps.k->n, launch == 1));
    if (uncovered) {
      opt.fused_plane = 0;
      lists[i].clear();
      st = build_passes(n, schedule, DFT3D_LAYOUT_NATURAL, opt, lists[i], ws, resolved);
      if (st != DFT3D_OK) return st;
    }
  }
  std::vector<const std::vector<Pass>*> ptrs;
  for (const auto& l : lists) ptrs.push_back(&l);
  const std::string s = batch_describe(ptrs, launch == 1);
  if (needed) *needed = s.size() + 1;
  if (buf && len > 0) {
    const size_t m = s.size() < len - 1 ? s.size() : len - 1;
    std::memcpy(buf, s.data(), m);
    buf[m] = '\0';
  }
  return DFT3D_OK;
}

int dft3d_plan(int64_t n0, int64_t n1, int64_t n2, int schedule, int layout,
               dft3d_plan_t* out) {
  if (!out) return DFT3D_ERR_INVALID_ARG;
  *out = nullptr;
  int st = validate(n0, n1, n2, schedule, layout);
  if (st != DFT3D_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return DFT3D_ERR_NO_DEVICE;
  }
  dft3d_plan_s* p = new (std::nothrow) dft3d_plan_s();
  if (!p) return DFT3D_ERR_OUT_OF_MEMORY;
  p->n[0] = n0;
  p->n[1] = n1;
  p->n[2] = n2;
  p->schedule = schedule;
  p->layout = layout;
  if (hipGetDevice(&p->device) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return DFT3D_ERR_HIP;
  }
  if (schedule == DFT3D_SCHED_AUTO && layout == DFT3D_LAYOUT_NATURAL) tune_lookup(p);
  st = rebuild(p);
  if (st != DFT3D_OK) {
    free_tables(p);
    delete p;
    return st;
  }
  *out = p;
  return DFT3D_OK;
}

int dft3d_plan_set_option(dft3d_plan_t p, int key, int64_t value) {
  if (!p) return DFT3D_ERR_INVALID_ARG;
  Options saved = p->opt;
  int st = apply_option(p->opt, key, value);
  if (st != DFT3D_OK) return st;
  st = rebuild(p);
  if (st != DFT3D_OK) {
    p->opt = saved;  // previous pass list stays in force
  } else {
    destroy_twin(p);        // rebuilt from the new options on demand
    batch_forget_plan(p);   // batched descriptors of the old pass list
  }
  return st;
}

int dft3d_plan_get_option(dft3d_plan_t p, int key, int64_t* value) {
  if (!p || !value) return DFT3D_ERR_INVALID_ARG;
  switch (key) {
    case DFT3D_OPT_PRECISION: *value = p->opt.precision; break;
    case DFT3D_OPT_TILE: *value = p->opt.tile; break;
    case DFT3D_OPT_XCD_REMAP: *value = p->opt.xcd_remap; break;
    case DFT3D_OPT_SPLIT_MAX: *value = p->opt.split_max; break;
    case DFT3D_OPT_NONTEMPORAL: *value = p->opt.nontemporal; break;
    case DFT3D_OPT_PERSISTENT: *value = p->opt.persistent; break;
    case DFT3D_OPT_SLAB_GROUP: *value = p->opt.slab_group; break;
    case DFT3D_OPT_FUSED_PLANE: *value = p->opt.fused_plane; break;
    case DFT3D_OPT_FUSED_AXES: *value = p->opt.fused_axes; break;
    case DFT3D_OPT_PENCIL_GROUP: *value = p->opt.pencil_group; break;
    case DFT3D_OPT_BATCH_LAUNCH: *value = p->opt.batch_launch; break;
    case DFT3D_OPT_MOVE_ONLY: *value = p->opt.move_only; break;
    case DFT3D_OPT_MFMA_LEAF: *value = p->opt.mfma_leaf; break;
    case DFT3D_OPT_RADICES: *value = (int64_t)p->opt.radices; break;
    case DFT3D_OPT_RADER: *value = p->opt.rader; break;
    case DFT3D_OPT_HALVES: *value = p->opt.halves; break;
    case DFT3D_OPT_PENCIL_ORDER: *value = p->opt.pencil_order; break;
    case DFT3D_OPT_NUM_PASSES: *value = (int64_t)p->passes.size(); break;
    default: return DFT3D_ERR_INVALID_ARG;
  }
  return DFT3D_OK;
}

int dft3d_workspace_size(dft3d_plan_t p, size_t* bytes) {
  if (!p || !bytes) return DFT3D_ERR_INVALID_ARG;
  *bytes = p->ws_need;
  return DFT3D_OK;
}

int dft3d_set_workspace(dft3d_plan_t p, void* dev_ptr, size_t bytes) {
  if (!p) return DFT3D_ERR_INVALID_ARG;
  if (!dev_ptr) {
    if (!p->ws_owned) {
      p->ws = nullptr;
      p->ws_bytes = 0;
    }
    return DFT3D_OK;
  }
  if (bytes < p->ws_need) return DFT3D_ERR_WORKSPACE_TOO_SMALL;
  free_workspace(p);
  p->ws = dev_ptr;
  p->ws_bytes = bytes;
  p->ws_owned = false;
  return DFT3D_OK;
}


int dft3d_execute(dft3d_plan_t p, const void* in, void* out, int sign, void* stream) {
  if (!p || !in || !out || (sign != -1 && sign != 1)) return DFT3D_ERR_INVALID_ARG;
  {
    const int st = check_device(p);
    if (st != DFT3D_OK) return st;
  }
  const size_t bytes = (size_t)(p->n[0] * p->n[1] * p->n[2]) * sizeof(float2);
  if (overlaps(in, out, bytes)) return DFT3D_ERR_INVALID_ARG;
  {
    const int st = ensure_workspace(p);
    if (st != DFT3D_OK) return st;
  }
  return execute_passes(p, in, out, sign, static_cast<hipStream_t>(stream), p->ws);
}

int dft3d_execute_batched(const dft3d_plan_t* plans, const void* const* in,
                          void* const* out, int count, int sign, void* stream) {
  if (count == 0) return DFT3D_OK;
  if (count < 0 || !plans || !in || !out || (sign != -1 && sign != 1))
    return DFT3D_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !in[i] || !out[i]) return DFT3D_ERR_INVALID_ARG;
    if (plans[i]->layout != DFT3D_LAYOUT_NATURAL || plans[i]->opt.precision != 0)
      return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    const int st = check_device(plans[i]);
    if (st != DFT3D_OK) return st;
    const size_t bytes =
        (size_t)(plans[i]->n[0] * plans[i]->n[1] * plans[i]->n[2]) * sizeof(float2);
    if (overlaps(in[i], out[i], bytes)) return DFT3D_ERR_INVALID_ARG;
  }
  return batch_execute(plans, in, out, count, sign, static_cast<hipStream_t>(stream));
}

int dft3d_destroy(dft3d_plan_t p) {
  if (!p) return DFT3D_OK;
  destroy_twin(p);
  batch_forget_plan(p);
  free_workspace(p);
  free_tables(p);
  delete p;
  return DFT3D_OK;
}

}  // extern "C"
