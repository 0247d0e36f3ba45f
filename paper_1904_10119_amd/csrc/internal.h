// Internal declarations shared by the host planner, the runtime and the
// kernel translation units of libdft3d.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace dft3d {

// How a pass reads or writes a tile of T pencils.
//   ROW: the pencil's own elements are contiguous (element stride 1), so
//        lanes run along the pencil;
//   COL: consecutive pencils are contiguous (pencil stride 1), so lanes run
//        across the T pencils of the tile and every element row is one
//        T * 8-byte segment.
enum Mode { MODE_ROW = 0, MODE_COL = 1 };

// Kernel arguments of one batched-1D-FFT pass.  Pencil b (0 <= b < B) is
// split into three bit fields b0 = b & m0, b1 = (b >> s0) & m1, b2 = b >> s1;
// element j of pencil b is read at  b2*is2 + b1*is1 + b0*is0 + j*ijs  and
// output k is written at  b2*os2 + b1*os1 + b0*os0 + k*oks  (complex64
// units).  With post_twiddle, output k of pencil b is multiplied by
// w_L^{(res * k) mod L}, res = (b >> res_shift) & res_mask, L = twp_mask + 1
// (the twiddle stage of eq. (3) / eq. (14)).
struct PassArgs {
  int64_t B;
  int64_t m0, m1;
  int32_t s0, s1;
  int64_t is0, is1, is2, ijs;
  int64_t os0, os1, os2, oks;
  int64_t res_mask, twp_mask;
  int32_t res_shift;
  int32_t conj_in, conj_out;  // inverse as conj(DFT(conj(x)))
  int32_t xcd_remap;          // 1: consecutive tiles on one XCD
};

using LaunchFn = hipError_t (*)(const PassArgs&, const float2* src, float2* dst,
                                const float2* tw, const float2* twp,
                                hipStream_t stream);

struct KernelInfo {
  int n;             // transform length
  int tile;          // pencils per workgroup
  int lmode, smode;  // Mode of the load and of the store
  int post_twiddle;  // 1: multiply outputs by the four-step twiddle
  int threads;       // workgroup size
  int lds_bytes;     // static LDS per workgroup
  LaunchFn launch;
  int persistent;    // 1: grid of resident workgroups walking all tiles
  int nontemporal;   // streaming accesses: 0 none, 1 loads and stores, 2 loads, 3 stores
  int precision = 0; // DFT3D_PREC_*: FP32 butterflies or split MFMA leaves
  int plane_rows = 0; // > 0: fused 2D DFT of (plane_rows, n) planes, one per workgroup
  int fused_axes = 0; // 1: volumetric V2 of one axis fused with V1 of the next (n = a);
                      // 2: the same with the finished axis left in the shuffled order;
                      // 3: inverse from the shuffled order (the transposed pass)
  int bluestein = 0;  // 1: one-pass Bluestein axis (length not a power of two, n = m)
  int mixed = 0;      // > 0: mixed-radix pass in LDS for lengths up to n (the variant)
  int fixed_n = 0;              // mixed-radix pass compiled for this one length, 0: any
  uint64_t fixed_code = 0;      // and its radix code
  int move_only = 0;  // 1: loads, LDS exchanges and stores of the pass with the radix
                      // stages (butterflies and twiddles) removed; 2: a plain copy
  int r0 = 0, r1 = 0, r2 = 0;   // FP32 pass kernels: the radix of each stage (1: none)
  int mfma_leaf = 0;  // split-precision MFMA passes: the leaf length (16 or 32)
  int rader = 0;      // > 0: Rader pass for prime lengths up to n - 1 (variant as mixed)
  int mfma_wide = 0;  // 1: MFMA one-tile pass with twice the default tile
  int halves = 0;     // 1: rotate-on-write pass of length n as two half-length
                      // transforms after a radix-2 split (halves_kernel.h)
};

// All compiled pass kernels.
const std::vector<KernelInfo>& kernel_registry();
// The move-only form (mode 1: radix stages removed; mode 2: a plain copy of
// the array) of an FP32 pass kernel, or null if none is compiled.
const KernelInfo* find_move_only_kernel(const KernelInfo* k, int mode);
const KernelInfo* find_kernel(int n, int tile, int lmode, int smode, int post_twiddle,
                              int persistent, int nontemporal);
// The two-halves pass of length n (halves_kernel.h) with the given load and
// store orders and form, or null if none is compiled.
const KernelInfo* find_halves_kernel(int n, int lmode, int smode, int persistent,
                                     int nontemporal, int move_only);
// The fused plane kernel for (n1, n2) planes, if compiled.
const KernelInfo* find_plane_kernel(int n1, int n2);
// Whether a mixed-radix kernel (variant 1: no 11 or 13 stages, composites
// 10 and 16 up to a tile length of 2048; variant 2: 11 and 13, no
// composites) runs every stage radix of a code.
bool mixed_kernel_runs(int variant, int nmax, uint64_t code);
// The mixed-radix pass kernel for length n, its radix code and the load
// and store modes, among those that run the code: the one with the given
// tile (pencils per workgroup) if compiled, else the first registered with
// the smallest tile length above n; null if none.
const KernelInfo* find_mixed_kernel(int64_t n, uint64_t code, int tile,
                                    int lmode = MODE_ROW, int smode = MODE_COL);
// Stage radices of a mixed-radix pass of length n, 8 bits per stage, first
// stage lowest; 0 if n has a prime factor above 13 or is 1.
uint64_t mixed_radix_code(int64_t n);
// The kernel variant a radix code needs.
int mixed_variant(uint64_t code);
// Whether a radix code is 0 or lists 1..8 stages of the mixed-radix
// kernel's radices (2, 3, 4, 5, 7, 8, 10, 11, 13, 16) whose product is at
// most 2048 and that a compiled mixed-radix kernel runs at that length.
bool radix_code_valid(uint64_t code);
// The product of a radix code's stages.
int64_t radix_code_length(uint64_t code);
// Whether a length is supported: every length 1..4096 (powers of two,
// mixed radix when the prime factors are at most 13, else Bluestein with a
// convolution length up to 8192).
bool length_supported(int64_t n);
// Whether n is prime with n - 1 free of prime factors above 13 and a Rader
// kernel runs it (the DFT of length n through two FFTs of length n - 1):
// one compiled for n, or with any_kernel also the generic one.
bool rader_length(int64_t n, bool any_kernel);
// The Rader kernel for prime length n (the radix code of n - 1), with the
// given tile if compiled, else the smallest tile length above n; null if none.
const KernelInfo* find_rader_kernel(int64_t n, int tile);
// Rader tables of prime length n: FFT_{n-1}(b) / (n - 1) with b[m] =
// w_n^(g^-m), FP64-built (n - 1 entries), then the generator powers g^j mod
// n (n - 1 32-bit integers, packed two per float2): rader_table_size slots.
int64_t rader_table_size(int64_t n);
void make_rader_tables(int64_t n, float2* out);
// The one-pass Bluestein axis kernel of convolution length m with the given
// tile, else the length's default tile; null if none is compiled.
const KernelInfo* find_bluestein_kernel(int m, int tile);
// The fused volumetric two-axis kernel for split factor a, if compiled
// (contig: V2 runs contiguous in memory; the persistent form if asked for;
// shuffled: the finished axis left in the shuffled order).
// kind: 1 natural, 2 shuffled forward, 3 inverse from the shuffled order
const KernelInfo* find_fused_axes_kernel(int a, int contig, int persistent, int kind);
// The split-precision MFMA pass kernel for a length and layout, if any
// (the persistent form when asked for and compiled, else the other form;
// the wide one-tile form where one is compiled, when the one-tile form or
// its tile is asked for), with leaves of length leaf (16 or 32; 0: the
// default for the length).
const KernelInfo* find_mfma_kernel(int n, int lmode, int smode, int precision,
                                   int persistent, int leaf, int tile = 0);
// The default MFMA leaf length of a pass length and split precision, and
// whether the persistent form is the default there.
int default_mfma_leaf(int n, int precision);
bool default_mfma_persistent(int n, int precision);

// Roots w_n^m = exp(-2 pi i m / n), m < n, computed in FP64 with exact
// octant reduction and rounded once to FP32 (eq. (4) entries).
void make_roots(int64_t n, float2* out);
// The same root in FP64: (cos, sin) of 2 pi m / n (before the sign).
void root_fp64(int64_t m, int64_t n, double& c, double& s);
// MFMA leaf operand tables for a precision (length-16 table, then the odd
// half table of the length-32 leaf; kLeafTableHalves 16-bit values).
constexpr int kLeafTableFloat2 = 2 * 3 * 2 * 64 * 8 / 4;  // as float2 slots
void make_leaf_table(int precision, unsigned short* out);
// Bluestein tables for a length n that is not a power of two: the chirp
// w[j] = exp(-pi i j^2 / n) (n entries) and the filter H / m, H = DFT_m of
// the wrapped conj(w[d]), d in (-n, n) (m entries), both from FP64.
int64_t bluestein_length(int64_t n);  // m: the power of two >= 2n - 1
// Stage twiddles of a mixed-radix pass (n - 1 entries): for the stage of
// radix R after ns = product of the earlier radices, entry
// (ns - 1) + (r - 1) ns + tm = w_{ns R}^{tm r} (r < R, tm < ns), from FP64.
void make_mixed_twiddles(int64_t n, uint64_t code, float2* out);
void make_chirp(int64_t n, float2* out);
void make_bluestein_filter(int64_t n, float2* out);

enum BufId { BUF_IN = 0, BUF_OUT = 1, BUF_WS = 2 };

struct Pass {
  const KernelInfo* k = nullptr;
  int src = BUF_IN, dst = BUF_OUT;
  PassArgs args{};
  int64_t in_off = 0, out_off = 0;  // element offsets into src / dst
  int64_t tw_len = 0;   // root table of the transform length (== k->n)
  int64_t twp_len = 0;  // post-twiddle table length, 0 if none
  int leaf = 0;         // precision of the MFMA leaf table the pass reads, 0: none
  int64_t bl_n = 0;     // Bluestein axis: the length n (tables: chirp, then filter)
  int64_t rader_n = 0;  // Rader axis: the prime length n
  // Which ends of the pass follow the plan's buffer chain (IN -> OUT/WS
  // alternation); the others keep the buffers the planner set.
  bool chain_src = true, chain_dst = true;
  std::string label;
};

struct Options {
  int precision = 0;
  int tile = 0;        // 0: default per pass
  int xcd_remap = 1;
  int split_max = 0;   // 0: default
  int nontemporal = 2; // 0 off, 1 on, 2 on for arrays above kStreamBytes
  int persistent = 1;  // use the persistent form where one exists
  int slab_group = -1; // slab: planes per row/column group (0 = all, -1 = auto)
  int fused_plane = 1; // slab: one fused 2D pass for planes that fit in LDS
  int fused_axes = 1;  // volumetric: V2 of an axis and V1 of the next in one pass
  int pencil_group = 0; // pencil: planes per group of the first two passes (0 = all, -1 = auto)
  int batch_launch = 0; // batched calls: 0 one launch per pass level, 1 one persistent launch
  int move_only = 0;    // 1: radix stages removed from every pass, 2: every pass a plain copy
  int mfma_leaf = 0;    // split-precision passes: leaf length 16 or 32, 0: default per length
  uint64_t radices = 0; // stage radices (8 bits each, first stage lowest) for the passes
                        // of their product's length, run by the mixed-radix kernel; 0: default
  int rader = 1;        // prime lengths with smooth n - 1: 0 Bluestein, 1 Rader where a
                        // kernel is compiled for n, 2 Rader also with the generic kernel
  int pencil_order = -1; // pencil schedule intermediates (powers of two, unsplit):
                         // 0 rotate (c2, c0, c1) each pass; 1 swap the two fastest
                         // axes on the first two passes; 2 cycle (A, B, C) ->
                         // (B, C, A) -> (C, A, B) -> (A, B, C); -1 automatic
  int halves = 1;       // rotate-on-write passes of length 2048 as two halves in
                        // 16-pencil tiles (1) or whole in 8-pencil tiles (0)
};

// Builds the pass list of a schedule.  Returns a dft3d status; on success
// fills passes and the workspace size in bytes.  from_layout = false gives
// the forward list (natural input, output in `layout` order); true gives
// the list that takes input in `layout` order to natural output, which the
// inverse of a shuffled plan runs (for the natural layout both coincide).
int build_passes(const int64_t n[3], int schedule, int layout, const Options& opt,
                 std::vector<Pass>& passes, size_t& ws_bytes, int& resolved_schedule,
                 bool from_layout = false);

// JSON description of a plan; inverse_passes (may be null) is listed as
// "inverse_passes" when given.
std::string describe_passes(const int64_t n[3], int schedule, int layout,
                            const std::vector<Pass>& passes,
                            const std::vector<Pass>* inverse_passes, size_t ws_bytes);

uint64_t next_plan_uid();

}  // namespace dft3d

// The plan behind the opaque dft3d_plan_t handle.
struct dft3d_plan_s {
  int64_t n[3] = {0, 0, 0};
  int schedule = 0;
  int resolved = 0;
  int layout = 0;
  dft3d::Options opt;
  std::vector<dft3d::Pass> passes;
  std::vector<int64_t> tw_off, twp_off;  // per pass, element offsets in tables
  // Shuffled layout only: the passes the inverse runs (input in shuffled
  // order, natural output) and their table offsets; empty otherwise.
  std::vector<dft3d::Pass> ipasses;
  std::vector<int64_t> itw_off, itwp_off;
  int device = -1;
  float2* tables = nullptr;
  size_t ws_need = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  uint64_t uid = 0;  // changes whenever the pass list is rebuilt
  int tuned = -1;    // AUTO plans: schedule chosen by the autotuner, -1 none
  // Plans with fused plane passes the batched plane kernel does not cover:
  // the same transform without them, built on first batched use.
  dft3d_plan_s* batch_twin = nullptr;
};

namespace dft3d {
// Allocates the plan-owned workspace if needed (dft3d status).
int ensure_workspace(dft3d_plan_s* p);
// DFT3D_OK if the current device is the plan's, else a status.
int check_device(const dft3d_plan_s* p);
// Enqueues the plan's passes on s with `ws` as the workspace (at least
// p->ws_need bytes, disjoint from in and out; may be null when the plan needs
// none).  Arguments are validated by the caller.  Allocates nothing.
int execute_passes(dft3d_plan_s* p, const void* in, void* out, int sign, hipStream_t s,
                   void* ws);
// Batched execution (batch.hip) and its cache upkeep.
int batch_execute(dft3d_plan_s* const* plans, const void* const* in,
                  void* const* out, int count, int sign, hipStream_t stream);
void batch_forget_plan(const dft3d_plan_s* p);
// AUTO plans: apply the autotuner's recorded choice for the shape, if any.
void tune_lookup(dft3d_plan_s* p);
// The plan whose passes the batched kernels run for p: p itself, or, when
// p has a fused plane pass the batched form (`persistent`: the one-launch
// form) does not cover, its twin without fused plane passes (created on
// first use; null on failure).
dft3d_plan_s* batch_view(dft3d_plan_s* p, bool persistent);
// Whether the batched plane kernels of a form cover (n1, n2) planes.
bool batch_runs_plane(int n1, int n2, bool persistent);
// Device-free description of how a batch of plans with these pass lists is
// laid out (JSON; see dft3d_batch_describe).
std::string batch_describe(const std::vector<const std::vector<Pass>*>& lists, bool persistent);
}  // namespace dft3d
