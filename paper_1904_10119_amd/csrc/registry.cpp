// Registry of the compiled pass kernels.
#include <algorithm>

#include "../../include/dft3d.h"
#include "internal.h"

namespace dft3d {

void register_kernels_small(std::vector<KernelInfo>& v);
void register_kernels_mid(std::vector<KernelInfo>& v);
void register_kernels_1k(std::vector<KernelInfo>& v);
void register_kernels_big(std::vector<KernelInfo>& v);
void register_kernels_mfma_a(std::vector<KernelInfo>& v);
void register_kernels_mfma_b(std::vector<KernelInfo>& v);
void register_kernels_mfma_c(std::vector<KernelInfo>& v);
void register_kernels_mfma_d(std::vector<KernelInfo>& v);
void register_kernels_mfma_e(std::vector<KernelInfo>& v);
void register_kernels_mfma_f(std::vector<KernelInfo>& v);
void register_kernels_plane(std::vector<KernelInfo>& v);
void register_kernels_fused(std::vector<KernelInfo>& v);
void register_kernels_bluestein(std::vector<KernelInfo>& v);
void register_kernels_mixed(std::vector<KernelInfo>& v);
void register_kernels_mixed_fixed(std::vector<KernelInfo>& v);
void register_kernels_rader(std::vector<KernelInfo>& v);
void register_kernels_rader_fixed(std::vector<KernelInfo>& v);
void register_kernels_halves(std::vector<KernelInfo>& v);

const std::vector<KernelInfo>& kernel_registry() {
  static const std::vector<KernelInfo> table = [] {
    std::vector<KernelInfo> v;
    register_kernels_small(v);
    register_kernels_mid(v);
    register_kernels_1k(v);
    register_kernels_big(v);
    register_kernels_mfma_a(v);
    register_kernels_mfma_b(v);
    register_kernels_mfma_c(v);
    register_kernels_mfma_d(v);
    register_kernels_mfma_e(v);
    register_kernels_mfma_f(v);
    register_kernels_plane(v);
    register_kernels_fused(v);
    register_kernels_bluestein(v);
    register_kernels_mixed(v);
    register_kernels_mixed_fixed(v);
    register_kernels_rader(v);
    register_kernels_rader_fixed(v);
    register_kernels_halves(v);
    return v;
  }();
  return table;
}

const KernelInfo* find_kernel(int n, int tile, int lmode, int smode, int post_twiddle,
                              int persistent, int nontemporal) {
  for (const KernelInfo& k : kernel_registry())
    if (k.n == n && k.tile == tile && k.lmode == lmode && k.smode == smode &&
        k.post_twiddle == post_twiddle && k.persistent == persistent &&
        k.nontemporal == nontemporal && k.precision == 0 && k.plane_rows == 0 &&
        k.fused_axes == 0 && k.bluestein == 0 && k.mixed == 0 && k.rader == 0 &&
        k.halves == 0 && k.move_only == 0)
      return &k;
  return nullptr;
}

const KernelInfo* find_halves_kernel(int n, int lmode, int smode, int persistent,
                                     int nontemporal, int move_only) {
  for (const KernelInfo& k : kernel_registry())
    if (k.halves && k.n == n && k.lmode == lmode && k.smode == smode &&
        k.persistent == persistent && k.nontemporal == nontemporal &&
        k.move_only == move_only)
      return &k;
  return nullptr;
}

const KernelInfo* find_move_only_kernel(const KernelInfo* k, int mode) {
  if (!k || k->precision || k->plane_rows || k->fused_axes || k->bluestein || k->mixed ||
      k->rader || k->move_only)
    return nullptr;
  if (k->halves && mode == 1)
    return find_halves_kernel(k->n, k->lmode, k->smode, k->persistent, k->nontemporal, 1);
  for (const KernelInfo& c : kernel_registry()) {
    if (c.move_only != mode || c.halves) continue;
    if (mode == 2 && c.n == k->n) return &c;
    if (mode == 1 && c.n == k->n && c.tile == k->tile && c.lmode == k->lmode &&
        c.smode == k->smode && c.post_twiddle == k->post_twiddle &&
        c.persistent == k->persistent && c.nontemporal == k->nontemporal &&
        c.r0 == k->r0 && c.r1 == k->r1 && c.r2 == k->r2)
      return &c;
  }
  return nullptr;
}

bool mixed_kernel_runs(int variant, int nmax, uint64_t code) {
  for (uint64_t c = code; c; c >>= 8) {
    const int r = (int)(c & 255);
    if (r == 11 || r == 13) {
      if (variant < 2) return false;
    } else if (r == 10 || r == 16) {  // composites: variant 1 up to 2048 only
      if (variant != 1 || nmax > 2048) return false;
    } else if (r != 2 && r != 3 && r != 4 && r != 5 && r != 7 && r != 8) {
      return false;
    }
  }
  return true;
}

const KernelInfo* find_mixed_kernel(int64_t n, uint64_t code, int tile, int lmode, int smode) {
  const int variant = mixed_variant(code);
  const KernelInfo* best = nullptr;
  if (tile <= 0)  // a kernel compiled for this length, code and modes, if any
    for (const KernelInfo& k : kernel_registry())
      if (k.mixed && k.fixed_n == n && k.fixed_code == code && k.lmode == lmode &&
          k.smode == smode)
        return &k;
  for (const KernelInfo& k : kernel_registry())
    if (k.mixed == variant && k.fixed_n == 0 && k.n > n && k.lmode == lmode &&
        k.smode == smode && mixed_kernel_runs(k.mixed, k.n, code)) {
      if (tile > 0 && k.tile == tile) return &k;  // the asked-for tile, if any
      if (!best || k.n < best->n) best = &k;      // else the first, smallest
    }
  return best;
}

uint64_t mixed_radix_code(int64_t n) {
  if (n < 2) return 0;
  const int64_t n0 = n;
  int count[14] = {0};
  for (int f : {2, 3, 5, 7, 11, 13})
    while (n % f == 0) {
      n /= f;
      ++count[f];
    }
  if (n != 1) return 0;
  // Composite radices (10 = 5 * 2, 16) only where the kernel without the
  // 11 and 13 stages runs them (lengths below 2048): fewer stages, each an
  // LDS round trip.
  const bool comp = count[11] == 0 && count[13] == 0 && n0 < 2048;
  // Odd radices first, then 10s, then powers of two: the first stage writes
  // its outputs at stride R in LDS, which an odd R spreads over every bank
  // (measured with SQ_LDS_BANK_CONFLICT at 1000^3); later stages write runs
  // of ns consecutive points.
  std::vector<int> radices;
  const int tens = comp ? std::min(count[5], count[2]) : 0;
  for (int f : {13, 11, 7, 5, 3})
    for (int i = 0; i < count[f] - (f == 5 ? tens : 0); ++i) radices.push_back(f);
  for (int i = 0; i < tens; ++i) radices.push_back(10);
  // the remaining power of two in as few stages as allowed (radix <= 16
  // with composites, else <= 8), the exponents spread evenly
  const int e = count[2] - tens, emax = comp ? 4 : 3;
  if (e > 0) {
    const int stages = (e + emax - 1) / emax;
    std::vector<int> ex(stages, e / stages);
    for (int i = 0; i < e % stages; ++i) ++ex[i];
    std::sort(ex.begin(), ex.end());
    for (int x : ex) radices.push_back(1 << x);
  }
  if (radices.size() > 8) return 0;
  uint64_t code = 0;
  for (size_t i = 0; i < radices.size(); ++i) code |= (uint64_t)radices[i] << (8 * i);
  return code;
}

int mixed_variant(uint64_t code) {
  for (uint64_t c = code; c; c >>= 8)
    if ((c & 255) == 11 || (c & 255) == 13) return 2;
  return 1;
}

int64_t radix_code_length(uint64_t code) {
  int64_t n = 1;
  for (uint64_t c = code; c; c >>= 8) n *= (int64_t)(c & 255);
  return n;
}

bool radix_code_valid(uint64_t code) {
  if (code == 0) return true;
  int stages = 0;
  int64_t n = 1;
  for (uint64_t c = code; c; c >>= 8) {
    const int r = (int)(c & 255);
    if (r != 2 && r != 3 && r != 4 && r != 5 && r != 7 && r != 8 && r != 10 && r != 11 &&
        r != 13 && r != 16)
      return false;  // a zero byte inside the code ends it early: rejected here too
    n *= r;
    if (++stages > 8 || n > 2048) return false;
  }
  // and a mixed-radix kernel runs the stages at that length
  return find_mixed_kernel(n, code, 0) != nullptr;
}

bool length_supported(int64_t n) { return n >= 1 && n <= 4096; }

namespace {
bool is_prime(int64_t n) {
  if (n < 2) return false;
  for (int64_t f = 2; f * f <= n; ++f)
    if (n % f == 0) return false;
  return true;
}
}  // namespace

const KernelInfo* find_rader_kernel(int64_t n, int tile) {
  const uint64_t code = mixed_radix_code(n - 1);
  if (!code) return nullptr;
  if (tile <= 0)  // a kernel compiled for this prime and code, if any
    for (const KernelInfo& k : kernel_registry())
      if (k.rader && k.fixed_n == n && k.fixed_code == code) return &k;
  const int variant = mixed_variant(code);
  const KernelInfo* best = nullptr;
  for (const KernelInfo& k : kernel_registry())
    if (k.rader == variant && k.fixed_n == 0 && k.n >= n + 1 &&
        mixed_kernel_runs(variant, k.n, code)) {
      if (tile > 0 && k.tile == tile) return &k;
      if (!best || k.n < best->n) best = &k;
    }
  return best;
}

bool rader_length(int64_t n, bool any_kernel) {
  if (n < 3 || !is_prime(n) || mixed_radix_code(n - 1) == 0) return false;
  const KernelInfo* k = find_rader_kernel(n, 0);
  return k && (any_kernel || k->fixed_n == n);
}

const KernelInfo* find_bluestein_kernel(int m, int tile) {
  const KernelInfo* first = nullptr;
  for (const KernelInfo& k : kernel_registry())
    if (k.bluestein && k.n == m) {
      if (k.tile == tile) return &k;
      if (!first) first = &k;
    }
  return first;
}

const KernelInfo* find_fused_axes_kernel(int a, int contig, int persistent, int kind) {
  const int mode = contig ? MODE_ROW : MODE_COL;
  const KernelInfo* other = nullptr;
  for (const KernelInfo& k : kernel_registry())
    if (k.fused_axes == kind && k.n == a && k.lmode == mode) {
      if (k.persistent == persistent) return &k;
      other = &k;
    }
  return other;
}

const KernelInfo* find_plane_kernel(int n1, int n2) {
  for (const KernelInfo& k : kernel_registry())
    if (k.plane_rows == n1 && k.n == n2) return &k;
  return nullptr;
}

// Measured on MI355X (pencil plans, same box): leaf 32 / leaf 16 time at
// 128^3, 256^3 and 4096 x 256 x 256 0.87 .. 0.97 in every split form, 64^3
// 1.10 .. 1.13 (64 = 32 * 2 against 16 * 4).  At lengths 1024 and 2048,
// with the cycled intermediate orders that split-precision pencil plans
// run, leaves of 16 are faster in every split form: 1024^3 bf16x6 10.57 ms
// (16) against 11.76 (32), bf16x9 11.43 / 12.83, fp16x3 12.19 / 12.46;
// 2048 x 1024 x 512 bf16x6 12.50 / 13.06, bf16x9 13.32 / 13.86, fp16x3
// 12.15 / 12.31.
int default_mfma_leaf(int n, int precision) {
  (void)precision;
  if (n == 128 || n == 256 || n == 4096) return 32;
  return 16;
}

// The persistent MFMA form (one workgroup per CU, next tile prefetched)
// against the one-tile form (two workgroups per CU, four waves per SIMD),
// cycled pencil orders: slower in every form measured (1024^3 fp16x3
// 14.46 against 12.19 ms, bf16x6 equal within 0.5 %; 2048 x 1024 x 512
// fp16x3 12.89 against 12.15), so the one-tile form is the default
// wherever both exist; the persistent form stays an option (nontemporal = 1
// with persistent on).
bool default_mfma_persistent(int n, int precision) {
  (void)n;
  (void)precision;
  return false;
}

const KernelInfo* find_mfma_kernel(int n, int lmode, int smode, int precision,
                                   int persistent, int leaf, int tile) {
  if (leaf == 0) leaf = default_mfma_leaf(n, precision);
  // the wide one-tile form where compiled (length 2048 rotated on write),
  // unless the persistent form or another tile is asked for
  if (tile > 0 || !persistent)
    for (const KernelInfo& k : kernel_registry())
      if (k.mfma_wide && k.n == n && k.lmode == lmode && k.smode == smode &&
          k.precision == precision && k.mfma_leaf == leaf && (tile <= 0 || k.tile == tile))
        return &k;
  const KernelInfo* other = nullptr;
  for (const KernelInfo& k : kernel_registry())
    if (!k.mfma_wide && k.n == n && k.lmode == lmode && k.smode == smode &&
        k.precision == precision && k.mfma_leaf == leaf) {
      if (k.persistent == persistent) return &k;
      other = &k;
    }
  return other;
}

int device_cu_count() {
  // One entry per device; CU counts do not change while the process runs.
  static int counts[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (counts[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    counts[dev] = n;
  }
  return counts[dev];
}

}  // namespace dft3d
