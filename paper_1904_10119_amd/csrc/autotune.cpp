// Autotuner: times candidate schedules and kernel options for one shape on
// the device and records the fastest as the choice of later AUTO plans of
// that shape.  Choices live in a process-wide table keyed by the device's
// architecture name and the shape, optionally mirrored to a text file
// (DFT3D_TUNE_CACHE): one line per entry,
//   arch n0 n1 n2 schedule tile xcd_remap split_max nontemporal persistent
//   slab_group pencil_group radices milliseconds
// Lines whose architecture differs from the current device are ignored.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dft3d.h"
#include "internal.h"

namespace dft3d {

namespace {

struct TuneEntry {
  int schedule;
  Options opt;
  double ms;
};

std::mutex g_tune_mutex;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string key_of(const std::string& arch, const int64_t n[3]) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s %lld %lld %lld", arch.c_str(), (long long)n[0],
                (long long)n[1], (long long)n[2]);
  return buf;
}

void load_file_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("DFT3D_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64];
  long long n0, n1, n2;
  int sched, tile, xcd, split, nt, pers, group, pgroup;
  unsigned long long radices;
  double ms;
  while (std::fscanf(f, "%63s %lld %lld %lld %d %d %d %d %d %d %d %d %llu %lf", arch, &n0, &n1,
                     &n2, &sched, &tile, &xcd, &split, &nt, &pers, &group, &pgroup, &radices,
                     &ms) == 14) {
    const int64_t n[3] = {n0, n1, n2};
    TuneEntry e;
    e.schedule = sched;
    e.opt.tile = tile;
    e.opt.xcd_remap = xcd;
    e.opt.split_max = split;
    e.opt.nontemporal = nt;
    e.opt.persistent = pers;
    e.opt.slab_group = group;
    e.opt.pencil_group = pgroup;
    e.opt.radices = radix_code_valid(radices) ? radices : 0;
    e.ms = ms;
    g_tune[key_of(arch, n)] = e;
  }
  std::fclose(f);
}

void save_file_locked() {
  const char* path = std::getenv("DFT3D_TUNE_CACHE");
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto& kv : g_tune) {
    const TuneEntry& e = kv.second;
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d %llu %.6f\n", kv.first.c_str(), e.schedule,
                 e.opt.tile, e.opt.xcd_remap, e.opt.split_max, e.opt.nontemporal,
                 e.opt.persistent, e.opt.slab_group, e.opt.pencil_group,
                 (unsigned long long)e.opt.radices, e.ms);
  }
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

}  // namespace

void tune_lookup(dft3d_plan_s* p) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  load_file_locked();
  const auto it = g_tune.find(key_of(arch_name(), p->n));
  if (it == g_tune.end()) return;
  const int precision = p->opt.precision;
  p->opt = it->second.opt;
  p->opt.precision = precision;
  p->tuned = it->second.schedule;
}

}  // namespace dft3d

using namespace dft3d;

extern "C" int dft3d_autotune(int64_t n0, int64_t n1, int64_t n2, const void* in, void* out,
                              void* stream, int* best_schedule, double* best_ms) {
  if (!in || !out) return DFT3D_ERR_INVALID_ARG;
  struct Cand {
    int schedule;
    int key;        // one option on top of the defaults (key 0: none)
    int64_t value;
  };
  static const Cand fixed_cands[] = {
      {DFT3D_SCHED_PENCIL, 0, 0},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_PERSISTENT, 0},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_PENCIL_GROUP, -1},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_SPLIT_MAX, 1024},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_SPLIT_MAX, 512},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_TILE, 8},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_TILE, 32},
      {DFT3D_SCHED_PENCIL, DFT3D_OPT_TILE, 64},
      {DFT3D_SCHED_SLAB, 0, 0},
      {DFT3D_SCHED_SLAB, DFT3D_OPT_PERSISTENT, 0},
      {DFT3D_SCHED_VOLUMETRIC, 0, 0},
  };
  std::vector<Cand> cands(std::begin(fixed_cands), std::end(fixed_cands));
  // radix sequences: for each axis length with a mixed-radix pass, the
  // default stage order reversed (powers of two first) and the power of two
  // in radix-4 stages, on the pencil schedule
  {
    const int64_t lens[3] = {n0, n1, n2};
    for (int d = 0; d < 3; ++d) {
      const int64_t n = lens[d];
      bool seen = false;
      for (int e = 0; e < d; ++e) seen = seen || lens[e] == n;
      if (seen || n < 2 || n > 2048 || (n & (n - 1)) == 0) continue;
      const uint64_t code = mixed_radix_code(n);
      if (!code) continue;
      std::vector<int> r;
      for (uint64_t c = code; c; c >>= 8) r.push_back((int)(c & 255));
      std::vector<uint64_t> alts;
      {  // reversed
        uint64_t a = 0;
        for (size_t i = 0; i < r.size(); ++i) a |= (uint64_t)r[r.size() - 1 - i] << (8 * i);
        alts.push_back(a);
      }
      {  // odd radices kept, the power of two as radix-4 stages (and one 2)
        std::vector<int> q;
        int64_t two = 1;
        for (int x : r) {
          if (x == 2 || x == 4 || x == 8 || x == 16) two *= x;
          else if (x == 10) { q.push_back(5); two *= 2; }
          else q.push_back(x);
        }
        while (two >= 4) { q.push_back(4); two /= 4; }
        if (two == 2) q.push_back(2);
        uint64_t a = 0;
        for (size_t i = 0; i < q.size() && i < 8; ++i) a |= (uint64_t)q[i] << (8 * i);
        if (q.size() <= 8) alts.push_back(a);
      }
      for (uint64_t a : alts)
        if (a != code && radix_code_valid(a) && radix_code_length(a) == n)
          cands.push_back(Cand{DFT3D_SCHED_PENCIL, DFT3D_OPT_RADICES, (int64_t)a});
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return DFT3D_ERR_HIP;
  }
  int best = -1;
  double best_time = 1e300;
  Options best_opt;
  int status = DFT3D_OK;
  for (const Cand& c : cands) {
    dft3d_plan_t p = nullptr;
    int st = dft3d_plan(n0, n1, n2, c.schedule, DFT3D_LAYOUT_NATURAL, &p);
    if (st != DFT3D_OK) {
      if (st == DFT3D_ERR_NO_DEVICE || st == DFT3D_ERR_UNSUPPORTED_SIZE ||
          st == DFT3D_ERR_INVALID_ARG) {
        status = st;
        break;
      }
      continue;
    }
    if (c.key && dft3d_plan_set_option(p, c.key, c.value) != DFT3D_OK) {
      dft3d_destroy(p);
      continue;
    }
    // warm up, then time a few executions; a candidate that cannot run
    // (e.g. no memory for its workspace) is skipped
    st = dft3d_execute(p, in, out, -1, stream);
    const int64_t points = n0 * n1 * n2;
    const int reps = points >= (int64_t(1) << 26) ? 3 : 10;
    float ms = 0.f;
    if (st == DFT3D_OK) {
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && st == DFT3D_OK; ++r) st = dft3d_execute(p, in, out, -1, stream);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = DFT3D_ERR_HIP;
    }
    if (st == DFT3D_OK && ms / reps < best_time) {
      best_time = ms / reps;
      best = p->resolved;
      best_opt = p->opt;
    }
    dft3d_destroy(p);
    (void)hipGetLastError();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != DFT3D_OK) return status;
  if (best < 0) return DFT3D_ERR_HIP;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    load_file_locked();
    const int64_t n[3] = {n0, n1, n2};
    best_opt.precision = DFT3D_PREC_FP32;
    g_tune[key_of(arch_name(), n)] = TuneEntry{best, best_opt, best_time};
    save_file_locked();
  }
  if (best_schedule) *best_schedule = best;
  if (best_ms) *best_ms = best_time;
  return DFT3D_OK;
}
