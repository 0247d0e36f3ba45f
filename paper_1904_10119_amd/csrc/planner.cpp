// Schedule planner: turns (n0, n1, n2, schedule) into a list of batched-1D
// FFT passes.  Pure host code; touches no device, so plans can be described
// and checked on a machine without a GPU.
//
//   PENCIL (eq. (8), Section 2.4): three passes; each transforms the
//     contiguous axis of the current (c0, c1, c2) array, seen as a (B, c2)
//     matrix, and writes the result transposed, (c2, B), so the data turns
//     xyz -> yzx -> zxy and is back in natural order after the third pass.
//   SLAB (eq. (6), Fig. 5): natural layout throughout; the 2D DFT of each
//     (n1, n2) plane (rows, then columns), then the 1D DFT along n0.
//   VOLUMETRIC (Fig. 9, eqs. (13)-(17)): natural layout; every axis of
//     length n = A * Bf is split four-step style: V1 = DFT_Bf over the
//     stride-A subsequences x[l + A k] of each residue l, times w_n^{l k'},
//     stored exchanged as T0[k'][l]; V2 = DFT_A over l, stored at
//     y[k' + Bf l'].
//   AUTO: below 256 MiB (arrays the Infinity Cache can hold between
//     passes) SLAB, whose planes of up to 128 x 128 points take one fused
//     pass; above it the pencil schedule (the cycled intermediate orders
//     where every axis is a power of two and unsplit), with axes longer than
//     a threshold split into V1 + V2 as in the volumetric schedule.
//   SHUFFLED layout (volumetric only; Section 2.4, Section 3.2): the forward
//     transform leaves out the final digit exchange of every split axis, so
//     natural entry y[k' + Bf l'] stays at position l' + A k' (V2 writes in
//     the layout it reads).  The inverse takes that order and returns
//     natural order: W1 = DFT_A over l' (contiguous in the shuffled order)
//     times w_n^{k' a}, then W2 = DFT_Bf over k' stored at a + A b.
#include <algorithm>
#include <cstdio>
#include <sstream>

#include "../../include/dft3d.h"
#include "internal.h"

namespace dft3d {

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

constexpr int kNoSplit = 62;  // bit position beyond any pencil index

// Default pencils per workgroup for a transform length.
int default_tile(int n) {
  switch (n) {
    case 1: case 2: case 4: case 8: case 16: return 256;
    case 32: return 128;
    case 64: return 64;
    case 128: return 32;
    case 256: return 32;
    case 512: return 16;
    case 1024: return 16;
    case 2048: return 8;
    default: return 4;
  }
}

// Arrays at least this large stream through HBM on every pass; below it the
// data may stay in the 256 MB Infinity Cache between passes.
constexpr int64_t kStreamBytes = int64_t(256) << 20;
// Largest group of planes the grouped pencil schedule keeps in the
// Infinity Cache between its first two passes.
constexpr int64_t kGroupBytes = int64_t(256) << 20;

// Kernel choice for one pass.  Measured on MI355X at 1024^3: the persistent
// prefetching kernels run best with streaming (non-temporal) accesses, the
// one-tile-per-workgroup kernels with ordinary ones.  Automatic mode uses
// the persistent form with streaming accesses for arrays that cannot stay
// in the caches, and the one-tile form with ordinary accesses otherwise.
const KernelInfo* pick_kernel(int n, int lmode, int smode, int tw, const Options& opt,
                              int64_t total_points) {
  struct Choice {
    int pers, nt;
  };
  Choice order[2];
  int nchoice = 0;
  if (opt.nontemporal == 2) {
    if (opt.persistent && total_points * 8 >= kStreamBytes) order[nchoice++] = {1, 1};
    order[nchoice++] = {0, 0};
  } else {
    if (opt.persistent) order[nchoice++] = {1, opt.nontemporal};
    order[nchoice++] = {0, opt.nontemporal};
  }
  // a two-halves kernel where one is compiled for the length and orders,
  // streaming and persistent under the same rule as the other passes,
  // except that the strided 2048 pass has one tile per workgroup only (its
  // persistent form measured slower: 5.42 against 5.29 ms per launch at
  // 2048 x 1024 x 512)
  if (opt.halves && tw == 0) {
    const bool big = total_points * 8 >= kStreamBytes;
    const int nt = opt.nontemporal == 2 ? (big ? 1 : 0) : opt.nontemporal;
    const int pers = opt.persistent && (opt.nontemporal != 2 || big) &&
                     !(n == 2048 && lmode == MODE_COL);
    if (const KernelInfo* k = find_halves_kernel(n, lmode, smode, pers, nt, 0))
      if (opt.tile <= 0 || opt.tile == k->tile) return k;
  }
  for (int c = 0; c < nchoice; ++c) {
    const int pers = order[c].pers, nt = order[c].nt;
    // the persistent rotate-on-write pass of length 512 in 32-pencil tiles
    // (256-byte row segments at one workgroup per CU: 3.50 against 3.68 ms
    // per launch at 2048 x 1024 x 512)
    if (opt.tile <= 0 && pers && n == 512 && lmode == MODE_ROW && smode == MODE_COL && !tw)
      if (const KernelInfo* k = find_kernel(n, 32, lmode, smode, tw, pers, nt)) return k;
    if (opt.tile > 0) {
      if (const KernelInfo* k = find_kernel(n, opt.tile, lmode, smode, tw, pers, nt)) return k;
    }
    if (const KernelInfo* k = find_kernel(n, default_tile(n), lmode, smode, tw, pers, nt))
      return k;
  }
  // any available tile for this length
  const int nt = order[nchoice - 1].nt;
  for (const KernelInfo& k : kernel_registry())
    if (k.n == n && k.lmode == lmode && k.smode == smode && k.post_twiddle == tw &&
        k.persistent == 0 && k.nontemporal == nt && k.precision == 0 && k.plane_rows == 0 &&
        k.fused_axes == 0 && k.bluestein == 0 && k.mixed == 0 && k.rader == 0 &&
        k.halves == 0 && k.move_only == 0)
      return &k;
  return nullptr;
}

struct Field {  // one bit field of the pencil index
  int64_t count;
  int64_t in_stride, out_stride;
};

// Whether a pencil-index decomposition needs the general form: a field
// whose count is not a power of two before the last field of count above 1.
bool general_fields(const Field* f, int nf) {
  while (nf > 1 && f[nf - 1].count == 1) --nf;
  for (int i = 0; i + 1 < nf; ++i)
    if (!is_pow2(f[i].count)) return true;
  return false;
}

// Fills the pencil-index decomposition of a pass from up to three fields,
// listed fastest first: bit fields, or where general_fields holds the
// general form (s0 = s1 = -1, m0 and m1 the counts of the first two fields;
// read only by the mixed-radix and Bluestein kernels, pencil_index.h).
void set_fields(PassArgs& a, const Field* f, int nf) {
  // trailing fields of count 1 after a count that is not a power of two
  // drop out (that count then ends the bit fields)
  for (int i = 0; i + 1 < nf; ++i)
    if (!is_pow2(f[i].count)) {
      while (nf > 1 && f[nf - 1].count == 1) --nf;
      break;
    }
  int64_t c0 = nf > 0 ? f[0].count : 1, c1 = nf > 1 ? f[1].count : 1;
  a.B = 1;
  for (int i = 0; i < nf; ++i) a.B *= f[i].count;
  if (general_fields(f, nf)) {
    a.s0 = a.s1 = -1;
    a.m0 = c0;
    a.m1 = c1;
    a.is0 = f[0].in_stride;
    a.os0 = f[0].out_stride;
    a.is1 = f[1].in_stride;
    a.os1 = f[1].out_stride;
    a.is2 = nf > 2 ? f[2].in_stride : 0;
    a.os2 = nf > 2 ? f[2].out_stride : 0;
    return;
  }
  a.s0 = nf > 1 ? ilog2(c0) : kNoSplit;
  a.m0 = nf > 1 ? c0 - 1 : (int64_t(1) << kNoSplit) - 1;
  a.is0 = nf > 0 ? f[0].in_stride : 0;
  a.os0 = nf > 0 ? f[0].out_stride : 0;
  a.s1 = nf > 2 ? a.s0 + ilog2(c1) : kNoSplit;
  a.m1 = nf > 2 ? c1 - 1 : (nf > 1 ? (int64_t(1) << (kNoSplit - a.s0)) - 1 : 0);
  a.is1 = nf > 1 ? f[1].in_stride : 0;
  a.os1 = nf > 1 ? f[1].out_stride : 0;
  a.is2 = nf > 2 ? f[2].in_stride : 0;
  a.os2 = nf > 2 ? f[2].out_stride : 0;
}

struct Builder {
  const Options& opt;
  std::vector<Pass>& passes;
  int64_t total_points;
  int status = DFT3D_OK;
  int nt_side = 0;  // > 0: prefer the persistent kernel with this one-sided NT form

  void add(int n, int lmode, int smode, int tw, const Field* f, int nf, int64_t ijs,
           int64_t oks, int64_t twp_len, int res_shift, int64_t res_mask,
           const std::string& label) {
    if (general_fields(f, nf)) {
      // pencil counts that are not powers of two (a shape with such an
      // axis): the power-of-two kernels read bit fields only, the
      // mixed-radix pass reads the general form and runs these lengths too
      if (tw) {
        status = DFT3D_ERR_UNSUPPORTED_SCHEDULE;
        return;
      }
      add_mixed(n, f, nf, ijs, oks, label + " mixed", lmode, smode);
      return;
    }
    if (opt.radices && radix_code_length(opt.radices) == n && !tw &&
        opt.precision == DFT3D_PREC_FP32 && !opt.move_only) {
      // a radix sequence asked for this length: the mixed-radix pass runs it
      add_mixed(n, f, nf, ijs, oks, label + " radices", lmode, smode);
      return;
    }
    const KernelInfo* k = nullptr;
    int leaf = 0;
    if (nt_side && opt.precision == DFT3D_PREC_FP32 && !tw)
      k = find_kernel(n, opt.tile > 0 ? opt.tile : default_tile(n), lmode, smode, 0, 1,
                      nt_side);
    if (!k && opt.precision != DFT3D_PREC_FP32 && !tw) {
      // split-precision leaves on the matrix cores where a kernel exists;
      // the one-tile form (two workgroups per CU, four waves per SIMD)
      // unless the persistent form measured faster for this length and
      // precision on arrays that stream through HBM (registry.cpp); with
      // streaming forced on (nontemporal = 1) the persistent form wherever
      // the persistent option is on
      const bool pers =
          opt.persistent &&
          (opt.nontemporal == 1 || (opt.nontemporal == 2 && total_points * 8 >= kStreamBytes &&
                                    default_mfma_persistent(n, opt.precision)));
      k = find_mfma_kernel(n, lmode, smode, opt.precision, pers, opt.mfma_leaf, opt.tile);
      // a length without leaves of the asked length keeps its default leaves
      if (!k && opt.mfma_leaf)
        k = find_mfma_kernel(n, lmode, smode, opt.precision, pers, 0, opt.tile);
      if (k) leaf = opt.precision;
    }
    if (!k) k = pick_kernel(n, lmode, smode, tw, opt, total_points);
    if (!k) {
      status = DFT3D_ERR_UNSUPPORTED_SIZE;
      return;
    }
    Pass p;
    p.k = k;
    p.leaf = leaf;
    set_fields(p.args, f, nf);
    p.args.ijs = ijs;
    p.args.oks = oks;
    p.args.xcd_remap = opt.xcd_remap;
    p.tw_len = n;
    p.twp_len = twp_len;
    if (tw) {
      p.args.res_shift = res_shift;
      p.args.res_mask = res_mask;
      p.args.twp_mask = twp_len - 1;
    }
    p.label = label;
    passes.push_back(p);
  }

  // Volumetric V2 of axis d fused with V1 of axis d-1 (fused_axes_kernel.h
  // documents the argument fields).
  void add_fused(const KernelInfo* k, const Field* f, int64_t row_step, int64_t sd,
                 int64_t b, int64_t n_prev, int a, const std::string& label) {
    Pass p;
    p.k = k;
    set_fields(p.args, f, 3);
    p.args.ijs = row_step;
    p.args.oks = sd;
    p.args.res_mask = b;
    p.args.twp_mask = n_prev - 1;
    p.args.xcd_remap = 0;
    p.tw_len = a;
    p.twp_len = n_prev;
    p.label = label;
    passes.push_back(p);
  }

  // One-pass Bluestein axis of length n (convolution length m) over the
  // pencils of fields f (bluestein.h documents the argument fields).
  void add_bluestein(int64_t n, const Field* f, int nf, int64_t ijs, int64_t oks,
                     const std::string& label) {
    const int64_t m = bluestein_length(n);
    const KernelInfo* k = find_bluestein_kernel((int)m, opt.tile);
    if (!k) {
      status = DFT3D_ERR_UNSUPPORTED_SIZE;
      return;
    }
    Pass p;
    p.k = k;
    set_fields(p.args, f, nf);
    p.args.ijs = ijs;
    p.args.oks = oks;
    p.args.res_mask = n;
    p.args.xcd_remap = opt.xcd_remap;
    p.tw_len = m;
    p.bl_n = n;
    p.label = label;
    passes.push_back(p);
  }

  // Rader pass of prime length n over the pencils of fields f (rader.h
  // documents the argument fields).
  void add_rader(int64_t n, const Field* f, int nf, int64_t ijs, int64_t oks,
                 const std::string& label) {
    const KernelInfo* k = find_rader_kernel(n, opt.tile);
    const uint64_t code = mixed_radix_code(n - 1);
    if (!k || !code) {
      status = DFT3D_ERR_UNSUPPORTED_SIZE;
      return;
    }
    Pass p;
    p.k = k;
    set_fields(p.args, f, nf);
    p.args.ijs = ijs;
    p.args.oks = oks;
    p.args.res_mask = n;
    p.args.twp_mask = (int64_t)code;
    p.args.xcd_remap = opt.xcd_remap;
    p.rader_n = n;
    p.label = label;
    passes.push_back(p);
  }

  // Mixed-radix pass of length n over the pencils of fields f
  // (mixed_kernel.h documents the argument fields).
  void add_mixed(int64_t n, const Field* f, int nf, int64_t ijs, int64_t oks,
                 const std::string& label, int lmode = MODE_ROW, int smode = MODE_COL) {
    const uint64_t code =
        opt.radices && radix_code_length(opt.radices) == n ? opt.radices : mixed_radix_code(n);
    const KernelInfo* k = find_mixed_kernel(n, code, opt.tile, lmode, smode);
    if (!k || !code) {
      status = DFT3D_ERR_UNSUPPORTED_SIZE;
      return;
    }
    Pass p;
    p.k = k;
    set_fields(p.args, f, nf);
    p.args.ijs = ijs;
    p.args.oks = oks;
    p.args.res_mask = n;
    p.args.twp_mask = (int64_t)code;
    p.args.xcd_remap = opt.xcd_remap;
    p.tw_len = n;
    p.label = label;
    passes.push_back(p);
  }

  // Fused 2D DFT of n0 contiguous (n1, n2) planes, in layout.
  void add_plane(const KernelInfo* k, int64_t n0, int64_t n1, int64_t n2,
                 const std::string& label) {
    Pass p;
    p.k = k;
    Field f[1] = {{n0, n1 * n2, n1 * n2}};
    set_fields(p.args, f, 1);
    p.args.ijs = 1;
    p.args.oks = 1;
    p.args.xcd_remap = 0;
    p.tw_len = n2;   // row roots
    p.twp_len = n1;  // column roots
    p.label = label;
    passes.push_back(p);
  }
};

// Four-step factor choice for a split axis: n = A * Bf with A the number of
// residues (the stride of the V1 subsequences) and Bf the V1 length.
void split_axis(int64_t n, int64_t& A, int64_t& Bf) {
  const int l = ilog2(n);
  A = int64_t(1) << ((l + 1) / 2);
  Bf = n / A;
}

// V1 + V2 of one axis in natural layout: the array is [outer][n][inner].
// With shuffled, V2 stores y[k' + Bf l'] at position l' + A k'.
void volumetric_v1(Builder& b, int64_t outer, int64_t n, int64_t inner, int axis) {
  int64_t A, Bf;
  split_axis(n, A, Bf);
  const int64_t slab = n * inner;
  char lab[64];
  {  // V1: pencils (o, l, c) with m = l * inner + c contiguous
    Field f[2] = {{A * inner, 1, 1}, {outer, slab, slab}};
    std::snprintf(lab, sizeof lab, "vol%d.V1 DFT%lld x%lld", axis, (long long)Bf,
                  (long long)(outer * A * inner));
    b.add((int)Bf, MODE_COL, MODE_COL, 1, f, 2, A * inner, A * inner, n,
          ilog2(inner), A - 1, lab);
  }
}

void volumetric_v2(Builder& b, int64_t outer, int64_t n, int64_t inner, int axis,
                   bool shuffled) {
  int64_t A, Bf;
  split_axis(n, A, Bf);
  const int64_t slab = n * inner;
  char lab[64];
  {  // V2: pencils (o, k', c); elements l at stride inner
    std::snprintf(lab, sizeof lab, "vol%d.V2%s DFT%lld x%lld", axis, shuffled ? " shuf" : "",
                  (long long)A, (long long)(outer * Bf * inner));
    if (shuffled && inner == 1) {  // output element l' at A k' + l'
      Field f[2] = {{Bf, A, A}, {outer, slab, slab}};
      b.add((int)A, MODE_ROW, MODE_ROW, 0, f, 2, 1, 1, 0, 0, 0, lab);
    } else if (shuffled) {
      Field f[3] = {{inner, 1, 1}, {Bf, A * inner, A * inner}, {outer, slab, slab}};
      b.add((int)A, MODE_COL, MODE_COL, 0, f, 3, inner, inner, 0, 0, 0, lab);
    } else if (inner == 1) {
      Field f[2] = {{Bf, A, 1}, {outer, slab, slab}};
      b.add((int)A, MODE_ROW, MODE_COL, 0, f, 2, 1, Bf, 0, 0, 0, lab);
    } else {
      Field f[3] = {{inner, 1, 1}, {Bf, A * inner, inner}, {outer, slab, slab}};
      b.add((int)A, MODE_COL, MODE_COL, 0, f, 3, inner, Bf * inner, 0, 0, 0, lab);
    }
  }
}

// The kernel for V2 of axis d and V1 of axis d - 1 in one pass, when
// a = A_d equals B_{d-1} and the tile fits the array; null otherwise.
const KernelInfo* fused_kernel_for(int64_t outer, int64_t n_prev, int64_t n, int64_t inner,
                                   int persistent, int kind) {
  int64_t A, Bf, Ap, Bp;
  split_axis(n, A, Bf);
  split_axis(n_prev, Ap, Bp);
  if (A != Bp) return nullptr;
  const int contig = inner == 1;
  const KernelInfo* k = find_fused_axes_kernel((int)A, contig, persistent, kind);
  if (!k) return nullptr;
  if (contig ? Bf % k->tile != 0 : (outer != 1 || inner % k->tile != 0)) return nullptr;
  return k;
}

// V2 of axis d and V1 of axis d - 1 in one pass where fused_kernel_for
// finds a kernel; returns false otherwise.  The array is
// [outer][n_prev][n][inner] with outer == 1 unless the V2 runs are
// contiguous (inner == 1).  kind 1: natural layout, 2: shuffled forward,
// 3: the inverse from the shuffled order (W2 of axis d - 1, then W1 of
// axis d, on the same tiles in place; twiddles of axis d, and with
// pre_twiddle those W1 of axis d - 1 left out).
bool volumetric_fused(Builder& b, int64_t outer, int64_t n_prev, int64_t n, int64_t inner,
                      int axis, int persistent, int kind, bool pre_twiddle = false) {
  int64_t A, Bf, Ap, Bp;
  split_axis(n, A, Bf);
  split_axis(n_prev, Ap, Bp);
  const int contig = inner == 1;
  const KernelInfo* k = fused_kernel_for(outer, n_prev, n, inner, persistent, kind);
  if (!k) return false;
  const bool shuffled = kind != 1;
  const int64_t KC = k->tile;
  const int64_t sd = inner, sprev = n * inner, so = n_prev * sprev;
  const int64_t twp_len = kind == 3 ? n : n_prev;
  char lab[64];
  if (kind == 3)
    std::snprintf(lab, sizeof lab, "vol%d.W2+vol%d.W1 DFT%lldx%lld", axis - 1, axis,
                  (long long)Bp, (long long)A);
  else
    std::snprintf(lab, sizeof lab, "vol%d.V2+vol%d.V1 DFT%lldx%lld%s", axis, axis - 1,
                  (long long)A, (long long)Bp, shuffled ? " shuffled" : "");
  // the run field: natural output k + b l' (runs KC apart at stride 1),
  // shuffled output a k' + l' where the run was read (same stride as in)
  if (contig) {
    Field f[3] = {{Bf / KC, KC * A * sd, shuffled ? KC * A * sd : KC * sd},
                  {Ap, sprev, sprev}, {outer, so, so}};
    b.add_fused(k, f, Ap * sprev, sd, Bf, twp_len, (int)A, lab);
  } else {
    Field f[3] = {{inner / KC, KC, KC}, {Ap, sprev, sprev},
                  {Bf, A * sd, shuffled ? A * sd : sd}};
    b.add_fused(k, f, Ap * sprev, sd, Bf, twp_len, (int)A, lab);
  }
  if (kind == 3 && pre_twiddle) {  // axis d - 1's first-half twiddle, from tw
    Pass& p = b.passes.back();
    p.args.res_shift = 1;
    p.args.res_mask = n_prev - 1;
    p.tw_len = n_prev;
  }
  return true;
}

// One axis of the inverse of a shuffled plan: input entry y[k' + Bf l'] at
// position l' + A k', natural output x[a + A b] at position a + A b:
//   x[a + A b] = sum_k' w_Bf^{k' b} w_n^{k' a} sum_l' w_A^{l' a} y[k' + Bf l']
// (forward roots; the inverse conjugates around the whole list).  W1 is the
// inner sum times the twiddle, W2 the outer sum.
// twiddle = false: the twiddle is left to the pass that runs W2 of the axis.
void volumetric_w1(Builder& b, int64_t outer, int64_t n, int64_t inner, int axis,
                   bool twiddle) {
  int64_t A, Bf;
  split_axis(n, A, Bf);
  const int64_t slab = n * inner;
  char lab[64];
  {  // W1: pencils (o, k', c), elements l' at A k' + l', outputs a there too
    std::snprintf(lab, sizeof lab, "vol%d.W1 DFT%lld x%lld%s", axis, (long long)A,
                  (long long)(outer * Bf * inner), twiddle ? "" : " untwiddled");
    const int tw = twiddle ? 1 : 0;
    const int64_t twl = twiddle ? n : 0;
    if (inner == 1) {
      Field f[2] = {{Bf, A, A}, {outer, slab, slab}};
      b.add((int)A, MODE_ROW, MODE_ROW, tw, f, 2, 1, 1, twl, 0, twiddle ? Bf - 1 : 0, lab);
    } else {
      Field f[3] = {{inner, 1, 1}, {Bf, A * inner, A * inner}, {outer, slab, slab}};
      b.add((int)A, MODE_COL, MODE_COL, tw, f, 3, inner, inner, twl,
            twiddle ? ilog2(inner) : 0, twiddle ? Bf - 1 : 0, lab);
    }
  }
}

void volumetric_w2(Builder& b, int64_t outer, int64_t n, int64_t inner, int axis) {
  int64_t A, Bf;
  split_axis(n, A, Bf);
  const int64_t slab = n * inner;
  char lab[64];
  {  // W2: pencils (o, a, c), elements k' at a + A k', outputs b at a + A b
    Field f[2] = {{A * inner, 1, 1}, {outer, slab, slab}};
    std::snprintf(lab, sizeof lab, "vol%d.W2 DFT%lld x%lld", axis, (long long)Bf,
                  (long long)(outer * A * inner));
    b.add((int)Bf, MODE_COL, MODE_COL, 0, f, 2, A * inner, A * inner, 0, 0, 0, lab);
  }
}

// One rotate-on-write step of the pencil schedule on a (c0, c1, c2) array:
// transform along c2 and write (c2, c0, c1).  With split, the c2 axis goes
// through V1 (natural) and a rotating V2.
void pencil_axis(Builder& b, const int64_t cur[3], bool split, int axis) {
  const int64_t n = cur[2], B = cur[0] * cur[1];
  char lab[64];
  if (!is_pow2(n) && mixed_radix_code(n)) {
    // prime factors <= 13 (mixed_kernel.h): one rotate-on-write pass
    Field f[1] = {{B, n, 1}};
    std::snprintf(lab, sizeof lab, "pencil%d DFT%lld mixed x%lld rot", axis, (long long)n,
                  (long long)B);
    b.add_mixed(n, f, 1, 1, B, lab);
    return;
  }
  if (!is_pow2(n) && b.opt.rader && rader_length(n, b.opt.rader == 2)) {
    // prime, n - 1 with factors <= 13 (rader.h): one rotate-on-write pass
    Field f[1] = {{B, n, 1}};
    std::snprintf(lab, sizeof lab, "pencil%d DFT%lld rader x%lld rot", axis, (long long)n,
                  (long long)B);
    b.add_rader(n, f, 1, 1, B, lab);
    return;
  }
  if (!is_pow2(n)) {
    // Bluestein (bluestein.h): the whole axis in one rotate-on-write pass
    Field f[1] = {{B, n, 1}};
    std::snprintf(lab, sizeof lab, "pencil%d DFT%lld via %lld x%lld rot", axis, (long long)n,
                  (long long)bluestein_length(n), (long long)B);
    b.add_bluestein(n, f, 1, 1, B, lab);
    return;
  }
  if (!split) {
    Field f[1] = {{B, n, 1}};
    std::snprintf(lab, sizeof lab, "pencil%d DFT%lld x%lld rot", axis, (long long)n,
                  (long long)B);
    b.add((int)n, MODE_ROW, MODE_COL, 0, f, 1, 1, B, 0, 0, 0, lab);
    return;
  }
  int64_t A, Bf;
  split_axis(n, A, Bf);
  {  // V1: pencils (o, l), elements x[o][l + A k]; T0[o][k'][l]
    Field f[2] = {{A, 1, 1}, {B, n, n}};
    std::snprintf(lab, sizeof lab, "pencil%d.V1 DFT%lld x%lld", axis, (long long)Bf,
                  (long long)(B * A));
    b.add((int)Bf, MODE_COL, MODE_COL, 1, f, 2, A, A, n, 0, A - 1, lab);
  }
  {  // V2 rotating: pencils (o fastest, k'); y[k' + Bf l'] goes to row
     // (k' + Bf l') of the (n, B) output
    Field f[2] = {{B, n, 1}, {Bf, A, B}};
    std::snprintf(lab, sizeof lab, "pencil%d.V2 DFT%lld x%lld rot", axis,
                  (long long)A, (long long)(B * Bf));
    b.add((int)A, MODE_ROW, MODE_COL, 0, f, 2, 1, Bf * B, 0, 0, 0, lab);
  }
}

// The pencil order a plan runs: the option, or automatically the cycle
// for split precision (1024^3 bf16x6 14.3 -> 12.2 ms, bf16x9 14.9 -> 11.4,
// 2048 x 1024 x 512 bf16x6 15.5 -> 13.1: the matrix-core passes' 64-byte
// row segments cost far less one row apart than one plane apart) and for
// FP32 arrays that stream through HBM (256 MiB and more) or have an axis of
// 2048 or more (2048 x 1024 x 512: 11.1 -> 10.6 ms; 4096 x 512 x 256:
// 7.17 -> 5.52; 1024^3: 10.62 -> 10.44 and 512^3 1.28 -> 1.26 with the
// one-tile kernels of add_cycled), else the rotation (256^3: 0.142 against
// 0.145 ms cycled).
int pencil_order(const int64_t n[3], const Options& opt) {
  if (opt.pencil_order >= 0) return opt.pencil_order;
  if (opt.precision != DFT3D_PREC_FP32) return 2;
  const bool long_axis = n[0] >= 2048 || n[1] >= 2048 || n[2] >= 2048;
  return long_axis || n[0] * n[1] * n[2] * 8 >= kStreamBytes ? 2 : 0;
}

// One rotate-on-write pass of the cycled order.  FP32 passes of length up
// to 1024 take the one-tile kernel (two workgroups' tiles in flight per CU
// instead of one persistent workgroup prefetching): measured in this order
// 1024^3 10.75 -> 10.44 ms, 512^3 1.29 -> 1.26 ms; the persistent form
// stays where streaming is forced on (nontemporal = 1) and for longer
// lengths (the 2048 pass as persistent halves).
void add_cycled(Builder& b, int len, const Field* f, int64_t oks, const char* lab) {
  if (b.opt.precision == DFT3D_PREC_FP32 && b.opt.nontemporal == 2 && b.nt_side == 0 &&
      len <= 1024) {
    Options one = b.opt;
    one.persistent = 0;
    Builder o{one, b.passes, b.total_points};
    o.add(len, MODE_ROW, MODE_COL, 0, f, 2, 1, oks, 0, 0, 0, lab);
    b.status = o.status;
    return;
  }
  b.add(len, MODE_ROW, MODE_COL, 0, f, 2, 1, oks, 0, 0, 0, lab);
}

// The pencil schedule in the other intermediate orders, on an (A, B, C)
// array of powers of two.  Order 1: the C pass writes (A, C, B) (output
// rows B apart instead of A B), the B pass reads pencils (a fastest, c) of
// that and writes (C, B, A) (rows A apart), and the A pass reads pencils
// (c fastest, b) and writes the natural (A, B, C).  Order 2: the cycle
// below.  Every pass loads whole pencils and stores rows of consecutive
// pencils, as the rotation does; only the intermediate orders differ.
void pencil_swapped(Builder& b, const int64_t n[3]) {
  const int64_t A = n[0], B = n[1], C = n[2];
  char lab[64];
  if (pencil_order(n, b.opt) == 2) {
    // every pass: tiles of pencils one plane apart, rows one row length
    // apart: (A, B, C) -> (B, C, A) -> (C, A, B) -> (A, B, C)
    {
      Field f[2] = {{A, B * C, 1}, {B, C, C * A}};
      std::snprintf(lab, sizeof lab, "pencil2 DFT%lld x%lld cyc", (long long)C,
                    (long long)(A * B));
      add_cycled(b, (int)C, f, A, lab);
    }
    if (b.status != DFT3D_OK) return;
    {
      Field f[2] = {{B, C * A, 1}, {C, A, A * B}};
      std::snprintf(lab, sizeof lab, "pencil0 DFT%lld x%lld cyc", (long long)A,
                    (long long)(B * C));
      add_cycled(b, (int)A, f, B, lab);
    }
    if (b.status != DFT3D_OK) return;
    {
      Field f[2] = {{C, A * B, 1}, {A, B, B * C}};
      std::snprintf(lab, sizeof lab, "pencil1 DFT%lld x%lld cyc", (long long)B,
                    (long long)(A * C));
      add_cycled(b, (int)B, f, C, lab);
    }
    return;
  }
  {
    Field f[2] = {{B, C, 1}, {A, B * C, C * B}};
    std::snprintf(lab, sizeof lab, "pencil2 DFT%lld x%lld swap", (long long)C, (long long)(A * B));
    b.add((int)C, MODE_ROW, MODE_COL, 0, f, 2, 1, B, 0, 0, 0, lab);
  }
  if (b.status != DFT3D_OK) return;
  {
    Field f[2] = {{A, C * B, 1}, {C, B, B * A}};
    std::snprintf(lab, sizeof lab, "pencil1 DFT%lld x%lld swap", (long long)B, (long long)(A * C));
    b.add((int)B, MODE_ROW, MODE_COL, 0, f, 2, 1, A, 0, 0, 0, lab);
  }
  if (b.status != DFT3D_OK) return;
  {
    Field f[2] = {{C, B * A, 1}, {B, A, C}};
    std::snprintf(lab, sizeof lab, "pencil0 DFT%lld x%lld rot", (long long)A, (long long)(B * C));
    b.add((int)A, MODE_ROW, MODE_COL, 0, f, 2, 1, B * C, 0, 0, 0, lab);
  }
}

// One pass of length n along an axis, in layout (element strides ijs, oks)
// over the pencils of fields f: the power-of-two pass kernels, else the
// mixed-radix pass (prime factors at most 13), else the one-pass Bluestein
// axis.  Used by the slab and volumetric schedules, whose passes keep the
// layout.
void axis_pass(Builder& b, int64_t n, int lmode, int smode, const Field* f, int nf,
               int64_t ijs, int64_t oks, const char* label) {
  char lab[96];
  if (is_pow2(n)) {
    b.add((int)n, lmode, smode, 0, f, nf, ijs, oks, 0, 0, 0, label);
  } else if (mixed_radix_code(n)) {
    std::snprintf(lab, sizeof lab, "%s mixed", label);
    b.add_mixed(n, f, nf, ijs, oks, lab, lmode, smode);
  } else if (b.opt.rader && rader_length(n, b.opt.rader == 2)) {
    std::snprintf(lab, sizeof lab, "%s rader", label);
    b.add_rader(n, f, nf, ijs, oks, lab);
  } else {
    std::snprintf(lab, sizeof lab, "%s via %lld", label, (long long)bluestein_length(n));
    b.add_bluestein(n, f, nf, ijs, oks, lab);
  }
}

// Grouped pencil schedule: planes of axis 0 taken G at a time through the
// first two passes, so that a group's intermediate (G n1 n2 points, about
// 256 MB) is read back by the second pass while it is still in the
// Infinity Cache; only the input read and the second pass's output write go
// to HBM.  For each group g (i0 = g G + i, i < G):
//   A_g: DFT along axis 2 of the (G, n1, n2) block of IN, rotated into the
//        group's own region of OUT as W[k2][i][i1];
//   B_g: DFT along axis 1 of W (pencils (i fastest, k2)), written to WS at
//        the full-array rotated place [k1][k2][g G + i];
// then one ordinary pencil pass along axis 0 from WS to OUT.  The passes of
// the two orders compute the same sums (eq. (8)); only the order in which
// the batches of 1D DFTs run differs.  Returns the group size, 0 if the
// shape does not take this form.
int64_t pencil_group_size(const int64_t n[3], const Options& opt, int64_t split_max) {
  if (opt.pencil_group == 0 || opt.precision != DFT3D_PREC_FP32) return 0;
  for (int d = 0; d < 3; ++d)
    if (!is_pow2(n[d])) return 0;
  if (n[0] < 2 || n[0] > split_max || n[1] > split_max || n[2] > split_max) return 0;
  const int64_t plane = n[1] * n[2];
  int64_t g;
  if (opt.pencil_group > 0) {
    g = std::min<int64_t>(opt.pencil_group, n[0]);
  } else {
    // automatic size: arrays that stream through HBM, groups of at most
    // 256 MB, and only where the one-sided streaming kernels exist for both
    // lengths.  Measured at 1024^3 on MI355X: 11.4 ms against 10.3 ms for
    // the ordinary schedule; a group's launch is eight tiles per workgroup
    // deep, and the unhidden first load and last store of each launch cost
    // more than the cache saves, so the option is off by default.
    if (n[0] * plane * 8 < kStreamBytes || opt.nontemporal != 2 || !opt.persistent) return 0;
    const int t2 = opt.tile > 0 ? opt.tile : default_tile((int)n[2]);
    const int t1 = opt.tile > 0 ? opt.tile : default_tile((int)n[1]);
    if (!find_kernel((int)n[2], t2, MODE_ROW, MODE_COL, 0, 1, 2) ||
        !find_kernel((int)n[1], t1, MODE_ROW, MODE_COL, 0, 1, 3))
      return 0;
    g = kGroupBytes / (plane * 8);
    if (g < 1) return 0;
  }
  int64_t p2 = 1;
  while (p2 * 2 <= g) p2 *= 2;
  return p2 < n[0] ? p2 : 0;  // one group is the ordinary schedule
}

void pencil_grouped(Builder& b, const int64_t n[3], int64_t G) {
  const int64_t n0 = n[0], n1 = n[1], n2 = n[2];
  char lab[80];
  for (int64_t g = 0; g < n0 / G && b.status == DFT3D_OK; ++g) {
    const int64_t base = g * G * n1 * n2;
    {  // A_g: pencils b = i n1 + i1 of the block; element k2 -> W[k2 (G n1) + b]
      Field f[1] = {{G * n1, n2, 1}};
      std::snprintf(lab, sizeof lab, "pencil2 DFT%lld x%lld rot group %lld", (long long)n2,
                    (long long)(G * n1), (long long)g);
      b.nt_side = 2;
      b.add((int)n2, MODE_ROW, MODE_COL, 0, f, 1, 1, G * n1, 0, 0, 0, lab);
      if (b.status != DFT3D_OK) break;
      Pass& p = b.passes.back();
      p.src = BUF_IN;
      p.dst = BUF_OUT;
      p.in_off = base;
      p.out_off = base;
      p.chain_src = p.chain_dst = false;
    }
    {  // B_g: pencils (i fastest, k2) of W; element k1 -> WS[k1 (n2 n0) + k2 n0 + g G + i]
      Field f[2] = {{G, n1, 1}, {n2, G * n1, n0}};
      std::snprintf(lab, sizeof lab, "pencil1 DFT%lld x%lld rot group %lld", (long long)n1,
                    (long long)(G * n2), (long long)g);
      b.nt_side = 3;
      b.add((int)n1, MODE_ROW, MODE_COL, 0, f, 2, 1, n2 * n0, 0, 0, 0, lab);
      if (b.status != DFT3D_OK) break;
      Pass& p = b.passes.back();
      p.src = BUF_OUT;
      p.dst = BUF_WS;
      p.in_off = base;
      p.out_off = g * G;
      p.chain_src = p.chain_dst = false;
    }
  }
  b.nt_side = 0;
  if (b.status != DFT3D_OK) return;
  Field f[1] = {{n1 * n2, n0, 1}};
  std::snprintf(lab, sizeof lab, "pencil0 DFT%lld x%lld rot", (long long)n0,
                (long long)(n1 * n2));
  b.add((int)n0, MODE_ROW, MODE_COL, 0, f, 1, 1, n1 * n2, 0, 0, 0, lab);
  if (b.status != DFT3D_OK) return;
  Pass& p = b.passes.back();
  p.src = BUF_WS;
  p.dst = BUF_OUT;
  p.chain_src = p.chain_dst = false;
}

// Buffers for a chain of passes from IN to OUT that never writes IN and
// never reads and writes the same buffer in one (not in-place-safe) pass.
void assign_chain(std::vector<Pass>& passes, size_t first, size_t& ws_needed_flag) {
  size_t cnt = 0;  // steps of the chain (passes whose destination follows it)
  for (size_t i = first; i < passes.size(); ++i) cnt += passes[i].chain_dst ? 1 : 0;
  // Alternate OUT / WS so that the last step writes OUT.
  int dst = (cnt % 2 == 1) ? BUF_OUT : BUF_WS;
  int src = BUF_IN;
  for (size_t i = first; i < passes.size(); ++i) {
    if (passes[i].chain_src) passes[i].src = src;
    if (!passes[i].chain_dst) continue;
    passes[i].dst = dst;
    if (dst == BUF_WS) ws_needed_flag = 1;
    src = dst;
    dst = (dst == BUF_OUT) ? BUF_WS : BUF_OUT;
  }
}

}  // namespace

int build_passes(const int64_t n[3], int schedule, int layout, const Options& given,
                 std::vector<Pass>& passes, size_t& ws_bytes, int& resolved,
                 bool from_layout) {
  passes.clear();
  ws_bytes = 0;
  // Move-only plans (the time breakdown of Section 4.3 on one device): the
  // schedule's passes with unfused kernels, each replaced by its form
  // without radix stages (1) or by a plain copy (2); FP32, natural layout,
  // powers of two.
  Options opt = given;
  if (opt.move_only) {
    if (opt.precision != DFT3D_PREC_FP32 || layout != DFT3D_LAYOUT_NATURAL)
      return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    opt.fused_plane = 0;
    opt.fused_axes = 0;
    opt.pencil_group = 0;
  }
  // powers of two up to 4096; other lengths through the mixed-radix or the
  // Bluestein pass (pencil schedule, FP32, natural layout only)
  bool any_other = false;
  for (int d = 0; d < 3; ++d) {
    if (!length_supported(n[d])) return DFT3D_ERR_UNSUPPORTED_SIZE;
    if (!is_pow2(n[d])) any_other = true;
  }
  if (schedule < DFT3D_SCHED_AUTO || schedule > DFT3D_SCHED_VOLUMETRIC)
    return DFT3D_ERR_INVALID_ARG;
  if (layout != DFT3D_LAYOUT_NATURAL && layout != DFT3D_LAYOUT_SHUFFLED)
    return DFT3D_ERR_INVALID_ARG;
  const bool shuffled = layout == DFT3D_LAYOUT_SHUFFLED;
  if (any_other && (shuffled || opt.precision != DFT3D_PREC_FP32 || opt.move_only))
    return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
  // only the volumetric schedule has a digit exchange to leave out
  if (shuffled && schedule != DFT3D_SCHED_VOLUMETRIC && schedule != DFT3D_SCHED_AUTO)
    return DFT3D_ERR_UNSUPPORTED_SCHEDULE;

  const int64_t total = n[0] * n[1] * n[2];
  Builder b{opt, passes, total};
  resolved = schedule;
  if (schedule == DFT3D_SCHED_AUTO)
    resolved = shuffled ? DFT3D_SCHED_VOLUMETRIC
                        : ((total * 8 < kStreamBytes && !any_other) ? DFT3D_SCHED_SLAB
                                                                    : DFT3D_SCHED_PENCIL);
  // Untuned AUTO splits only 4096-long axes (a 4096 pencil leaves tiles of
  // four pencils); measured at 2048x1024x512, the 2048 pass beats its split.
  const int64_t split_max =
      opt.split_max > 0 ? opt.split_max
                        : (schedule == DFT3D_SCHED_AUTO ? 2048 : int64_t(1) << 20);

  size_t need_ws = 0;
  const int64_t group = resolved == DFT3D_SCHED_PENCIL && !shuffled
                            ? pencil_group_size(n, opt, split_max)
                            : 0;
  if (group > 0) {
    pencil_grouped(b, n, group);
    need_ws = 1;
  } else if (resolved == DFT3D_SCHED_PENCIL && pencil_order(n, opt) > 0 && is_pow2(n[0]) &&
             is_pow2(n[1]) && is_pow2(n[2]) && n[0] <= split_max && n[1] <= split_max &&
             n[2] <= split_max) {
    pencil_swapped(b, n);
    assign_chain(passes, 0, need_ws);
  } else if (resolved == DFT3D_SCHED_PENCIL) {
    int64_t cur[3] = {n[0], n[1], n[2]};
    for (int step = 0; step < 3; ++step) {
      const int axis = 2 - step;
      // a split needs power-of-two pencil counts (bit-field pencil indices)
      const bool split = is_pow2(cur[2]) && cur[2] > split_max && cur[2] >= 4 &&
                         is_pow2(cur[0] * cur[1]);
      pencil_axis(b, cur, split, axis);
      if (b.status != DFT3D_OK) break;
      const int64_t c2 = cur[2];
      cur[2] = cur[1];
      cur[1] = cur[0];
      cur[0] = c2;
    }
    assign_chain(passes, 0, need_ws);
  } else if (resolved == DFT3D_SCHED_SLAB) {
    // 2D DFT of every (n1, n2) plane: rows (axis 2) IN -> OUT, columns
    // (axis 1) in place.  Planes go in groups, rows then columns per group,
    // so that a group written by the row pass can still be in the Infinity
    // Cache when its column pass reads it.  Then axis 0 in place.
    const int64_t plane = n[1] * n[2];
    int64_t group = opt.slab_group;
    if (group < 0) group = 0;  // automatic: all planes in one pass each
    if (group == 0 || group > n[0]) group = n[0];
    while (n[0] % group) --group;
    char lab[64];
    // planes that fit in one workgroup's LDS: rows and columns in one pass
    const KernelInfo* pk = (opt.fused_plane && opt.precision == DFT3D_PREC_FP32 &&
                            group == n[0])
                               ? find_plane_kernel((int)n[1], (int)n[2])
                               : nullptr;
    if (pk) {
      std::snprintf(lab, sizeof lab, "slab.plane DFT%lldx%lld planes %lld", (long long)n[1],
                    (long long)n[2], (long long)n[0]);
      b.add_plane(pk, n[0], n[1], n[2], lab);
      passes.back().src = BUF_IN;
      passes.back().dst = BUF_OUT;
    }
    for (int64_t g0 = 0; g0 < n[0] && !pk; g0 += group) {
      {
        Field f[1] = {{group * n[1], n[2], n[2]}};
        std::snprintf(lab, sizeof lab, "slab.rows DFT%lld planes %lld+%lld", (long long)n[2],
                      (long long)g0, (long long)group);
        axis_pass(b, n[2], MODE_ROW, MODE_ROW, f, 1, 1, 1, lab);
        if (b.status != DFT3D_OK) break;
        passes.back().src = BUF_IN;
        passes.back().dst = BUF_OUT;
        passes.back().in_off = passes.back().out_off = g0 * plane;
      }
      {
        Field f[2] = {{n[2], 1, 1}, {group, plane, plane}};
        std::snprintf(lab, sizeof lab, "slab.cols DFT%lld planes %lld+%lld", (long long)n[1],
                      (long long)g0, (long long)group);
        axis_pass(b, n[1], MODE_COL, MODE_COL, f, 2, n[2], n[2], lab);
        if (b.status != DFT3D_OK) break;
        passes.back().src = passes.back().dst = BUF_OUT;
        passes.back().in_off = passes.back().out_off = g0 * plane;
      }
    }
    if (b.status == DFT3D_OK) {
      Field f[1] = {{plane, 1, 1}};
      std::snprintf(lab, sizeof lab, "slab.depth DFT%lld", (long long)n[0]);
      axis_pass(b, n[0], MODE_COL, MODE_COL, f, 1, plane, plane, lab);
      if (b.status == DFT3D_OK) passes.back().src = passes.back().dst = BUF_OUT;
    }
  } else {  // VOLUMETRIC
    // FP32 plans fuse V2 of an axis with V1 of the next where the split
    // factors match (four passes instead of six for 256^3, 1024^3)
    // (the shuffled forward list too: its fused passes leave the finished
    // axis in digit order; the inverse from the shuffled order runs the
    // transposed passes in reverse order, W1 of axis 0 first)
    const bool fuse = opt.fused_axes && opt.precision == DFT3D_PREC_FP32 && !any_other;
    // the persistent fused form only when streaming is forced on: at 1024^3
    // it measured no faster (15.0 vs 14.7 ms for the schedule), the one-tile
    // form's workgroup turnover already overlaps the phases
    const int fpers = opt.persistent && opt.nontemporal == 1;
    int pending = -1;  // axis whose V2 (W2 from the shuffled order) is still to come
    auto dims = [&n](int axis, int64_t& outer, int64_t& inner) {
      outer = 1;
      inner = 1;
      for (int d = 0; d < axis; ++d) outer *= n[d];
      for (int d = axis + 1; d < 3; ++d) inner *= n[d];
    };
    auto in_layout = [&](int axis, int64_t outer, int64_t inner) {
      // too short to split (its shuffled order is natural), or not a power
      // of two: one pass in layout
      char lab[64];
      std::snprintf(lab, sizeof lab, "vol%d DFT%lld", axis, (long long)n[axis]);
      if (inner == 1) {
        Field f[1] = {{outer, n[axis], n[axis]}};
        axis_pass(b, n[axis], MODE_ROW, MODE_ROW, f, 1, 1, 1, lab);
      } else {
        Field f[2] = {{inner, 1, 1}, {outer, n[axis] * inner, n[axis] * inner}};
        axis_pass(b, n[axis], MODE_COL, MODE_COL, f, 2, inner, inner, lab);
      }
    };
    auto flush = [&]() {
      if (pending < 0) return;
      int64_t o, in;
      dims(pending, o, in);
      volumetric_v2(b, o, n[pending], in, pending, shuffled);
      pending = -1;
    };
    if (shuffled && from_layout) {
      // inverse from the shuffled order: per split axis W1 then W2; W2 of
      // an axis and W1 of the next inner one share a pass where the split
      // factors match
      auto flush_w2 = [&]() {
        if (pending < 0) return;
        int64_t o, in;
        dims(pending, o, in);
        volumetric_w2(b, o, n[pending], in, pending);
        pending = -1;
      };
      auto split_at = [&](int axis) {
        int64_t o, in;
        dims(axis, o, in);
        return n[axis] >= 4 && is_pow2(n[axis]) && is_pow2(in);
      };
      // W2 of axis e (split) and W1 of axis e + 1 share a pass
      auto fuses = [&](int e) {
        if (!fuse || e + 1 > 2 || !split_at(e) || !split_at(e + 1)) return false;
        int64_t po, pin, o, in;
        dims(e, po, pin);
        dims(e + 1, o, in);
        return fused_kernel_for(po, n[e], n[e + 1], in, fpers, 3) != nullptr;
      };
      bool owed = false;  // the pending axis's W1 twiddle is still to apply
      for (int axis = 0; axis < 3; ++axis) {
        int64_t outer = 1, inner = 1;
        dims(axis, outer, inner);
        if (!split_at(axis)) {
          flush_w2();
          in_layout(axis, outer, inner);
          continue;
        }
        if (pending >= 0 && pending == axis - 1 && fuses(pending)) {
          int64_t po, pin;
          dims(pending, po, pin);
          // the array as [po][n[pending]][n[axis]][inner]
          if (!volumetric_fused(b, po, n[pending], n[axis], inner, axis, fpers, 3, owed)) {
            b.status = DFT3D_ERR_UNSUPPORTED_SCHEDULE;  // fuses() said it would
            break;
          }
          pending = axis;
          owed = false;
          continue;
        }
        flush_w2();
        // a W1 whose W2 will share a pass with the next axis leaves its
        // twiddle to that pass (a row twiddle uniform over the workgroup)
        owed = fuses(axis);
        volumetric_w1(b, outer, n[axis], inner, axis, !owed);
        pending = axis;
      }
      flush_w2();
    } else {
      for (int axis = 2; axis >= 0; --axis) {
        int64_t outer = 1, inner = 1;
        dims(axis, outer, inner);
        // a four-step split needs power-of-two bit fields: the axis and the
        // axes after it (the residue of the twiddle stage is a bit field of
        // the pencil index); other axes run as one pass in layout
        const bool split = n[axis] >= 4 && is_pow2(n[axis]) && is_pow2(inner);
        if (split) {
          if (pending == axis + 1 && fuse && n[pending] >= 4) {
            int64_t po, pin;
            dims(pending, po, pin);
            // the pending axis's outer dimensions are [outer][n[axis]]
            if (volumetric_fused(b, outer, n[axis], n[pending], pin, pending, fpers,
                                 shuffled ? 2 : 1)) {
              pending = axis;
              continue;
            }
          }
          flush();
          volumetric_v1(b, outer, n[axis], inner, axis);
          pending = axis;
          continue;
        }
        flush();
        in_layout(axis, outer, inner);
      }
      flush();
    }
    assign_chain(passes, 0, need_ws);
  }
  if (b.status != DFT3D_OK) {
    passes.clear();
    return b.status;
  }
  if (opt.move_only) {
    if (any_other) {
      passes.clear();
      return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
    }
    for (Pass& ps : passes) {
      const KernelInfo* m = find_move_only_kernel(ps.k, opt.move_only);
      if (!m) {
        passes.clear();
        return DFT3D_ERR_UNSUPPORTED_SCHEDULE;
      }
      ps.k = m;
      ps.label += opt.move_only == 1 ? " move-only" : " copy";
    }
  }
  ws_bytes = need_ws ? (size_t)total * 8 : 0;
  return DFT3D_OK;
}

namespace {
void describe_list(std::ostringstream& os, const std::vector<Pass>& passes) {
  static const char* kBuf[] = {"in", "out", "ws"};
  os << "[";
  for (size_t i = 0; i < passes.size(); ++i) {
    const Pass& p = passes[i];
    if (i) os << ",";
    os << "{\"label\":\"" << p.label << "\",\"n\":" << p.k->n << ",\"tile\":" << p.k->tile
       << ",\"load\":\"" << (p.k->lmode == MODE_ROW ? "row" : "col") << "\",\"store\":\""
       << (p.k->smode == MODE_ROW ? "row" : "col") << "\",\"post_twiddle\":"
       << p.k->post_twiddle << ",\"persistent\":" << p.k->persistent
       << ",\"nontemporal\":" << p.k->nontemporal << ",\"precision\":" << p.k->precision
       << ",\"plane_rows\":" << p.k->plane_rows << ",\"fused_axes\":" << p.k->fused_axes
       << ",\"bluestein\":" << p.k->bluestein << ",\"bl_n\":" << p.bl_n
       << ",\"mixed\":" << p.k->mixed << ",\"fixed_n\":" << p.k->fixed_n
       << ",\"rader\":" << p.k->rader << ",\"rader_n\":" << p.rader_n
       << ",\"halves\":" << p.k->halves
       << ",\"move_only\":" << p.k->move_only << ",\"radices\":[";
    if (p.k->mixed || p.k->rader) {  // the stage radices (of n - 1 for Rader), first first
      bool first = true;
      for (uint64_t c = (uint64_t)p.args.twp_mask; c; c >>= 8, first = false)
        os << (first ? "" : ",") << (c & 255);
    } else if (p.k->r0 > 0) {  // FP32 pass kernels: their radix stages
      os << p.k->r0;
      if (p.k->r1 > 1) os << "," << p.k->r1;
      if (p.k->r2 > 1) os << "," << p.k->r2;
    } else if (p.k->mfma_leaf) {  // MFMA passes: leaf stages, then the VALU rest
      int n = p.k->n;
      bool first = true;
      for (; n >= p.k->mfma_leaf; n /= p.k->mfma_leaf, first = false)
        os << (first ? "" : ",") << p.k->mfma_leaf;
      if (n > 1) os << "," << n;
    }
    os << "]"
       << ",\"mfma_leaf\":" << p.k->mfma_leaf << ",\"threads\":" << p.k->threads
       << ",\"lds_bytes\":" << p.k->lds_bytes << ",\"pencils\":" << p.args.B
       << ",\"src\":\"" << kBuf[p.src] << "\",\"dst\":\"" << kBuf[p.dst] << "\""
       << ",\"in_off\":" << p.in_off << ",\"out_off\":" << p.out_off
       << ",\"args\":{\"B\":" << p.args.B << ",\"m0\":" << p.args.m0
       << ",\"m1\":" << p.args.m1 << ",\"s0\":" << p.args.s0 << ",\"s1\":" << p.args.s1
       << ",\"is\":[" << p.args.is0 << "," << p.args.is1 << "," << p.args.is2 << "]"
       << ",\"os\":[" << p.args.os0 << "," << p.args.os1 << "," << p.args.os2 << "]"
       << ",\"ijs\":" << p.args.ijs << ",\"oks\":" << p.args.oks
       << ",\"res_shift\":" << p.args.res_shift << ",\"res_mask\":" << p.args.res_mask
       << ",\"twp_len\":" << p.twp_len << ",\"tw_len\":" << p.tw_len << "}}";
  }
  os << "]";
}
}  // namespace

std::string describe_passes(const int64_t n[3], int schedule, int layout,
                            const std::vector<Pass>& passes,
                            const std::vector<Pass>* inverse_passes, size_t ws_bytes) {
  static const char* kSched[] = {"auto", "slab", "pencil", "volumetric"};
  std::ostringstream os;
  os << "{\"shape\":[" << n[0] << "," << n[1] << "," << n[2] << "],\"schedule\":\""
     << kSched[schedule] << "\",\"layout\":\""
     << (layout == DFT3D_LAYOUT_SHUFFLED ? "shuffled" : "natural")
     << "\",\"workspace_bytes\":" << ws_bytes << ",\"passes\":";
  describe_list(os, passes);
  if (inverse_passes) {
    os << ",\"inverse_passes\":";
    describe_list(os, *inverse_passes);
  }
  os << "}";
  return os.str();
}

}  // namespace dft3d
