/*
 * dft3d -- 3D complex DFT on one AMD Instinct MI355X (gfx950).
 *
 * Computes the 3D DFT (Section 2.1, eqs. (1)-(2); Section 2.3, eqs. (6)-(8))
 *
 *   y[k0,k1,k2] = sum_{i0,i1,i2} x[i0,i1,i2] w_{n0}^{i0 k0} w_{n1}^{i1 k1}
 *                                            w_{n2}^{i2 k2},
 *   w_n = exp(sign * 2 pi i / n),
 *
 * as passes of batched 1D FFTs with layout changes between them.  The
 * paper's decompositions become on-device schedules:
 *   SLAB        2D DFT of every (n1, n2) plane, then a 1D DFT along n0
 *               (eq. (6), Fig. 5);
 *   PENCIL      three passes of 1D DFTs, each writing its output rotated so
 *               that the next axis is contiguous, xyz -> yzx -> zxy -> xyz
 *               (eq. (8), Fig. 6, Section 2.4);
 *   VOLUMETRIC  every axis of length n = a b split four-step style (eq. (3),
 *               eqs. (13)-(17)): batched DFT_b over the stride-a subsequences
 *               with the twiddle of eq. (4) and an exchanging store, then
 *               batched DFT_a (Fig. 9, Section 3.2);
 *   AUTO        a per-shape choice: the autotuner's measured choice when
 *               one is recorded, otherwise SLAB below 256 MiB (arrays the
 *               Infinity Cache can hold) and PENCIL from 256 MiB on.
 *
 * Data: complex64 = two IEEE binary32 (re, im), interleaved, 8 bytes per
 * point; C order (n0, n1, n2), n2 contiguous; device pointers, 16-byte
 * aligned.  Forward is sign = -1 and inverse sign = +1; neither is scaled,
 * so inverse(forward(x)) = n0 n1 n2 x.
 *
 * Every call returns a status (DFT3D_OK = 0, errors negative).  Argument
 * errors are detected before any work is enqueued; after any error nothing
 * is leaked and output handles are set to NULL.  Plans are not thread-safe: one plan is used from one host
 * thread and one stream at a time; distinct plans are independent.
 */
#ifndef DFT3D_H
#define DFT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dft3d_plan_s* dft3d_plan_t;

/* Schedules (the paper's decompositions, Section 2.3/2.4 and Fig. 9). */
enum dft3d_schedule {
  DFT3D_SCHED_AUTO = 0,
  DFT3D_SCHED_SLAB = 1,
  DFT3D_SCHED_PENCIL = 2,
  DFT3D_SCHED_VOLUMETRIC = 3
};

/* Layouts of the transformed data.  NATURAL is C order (n0, n1, n2) on both
 * sides.  SHUFFLED (VOLUMETRIC and AUTO schedules only, which then resolves
 * to VOLUMETRIC; others return DFT3D_ERR_UNSUPPORTED_SCHEDULE) drops the
 * final digit exchange of every split axis (Section 2.4, Section 3.2): along
 * an axis of length n >= 4 split n = a b with a = 2^ceil(log2(n) / 2),
 * the transformed entry of natural index k' + b l' (k' < b, l' < a) is kept
 * at position l' + a k'; axes shorter than 4 stay in natural order.  The
 * forward transform (sign -1) takes natural input and writes this order;
 * the inverse (sign +1) takes input in this order and writes natural order,
 * so a pointwise product between the two (a convolution) needs neither
 * exchange.  Batched execution accepts NATURAL plans only. */
enum dft3d_layout { DFT3D_LAYOUT_NATURAL = 0, DFT3D_LAYOUT_SHUFFLED = 1 };

/* Leaf arithmetic.  FP32 runs every butterfly in binary32 with twiddles
 * generated in FP64 and rounded once.  The split forms run leaf DFTs of
 * length 16 or 32 as real GEMMs on the matrix cores with operands split
 * into bf16 / fp16 terms and FP32 accumulation; X1 forms use a single term
 * and are not accurate to FP32 (reported, never a parity claim). */
enum dft3d_precision {
  DFT3D_PREC_FP32 = 0,
  DFT3D_PREC_BF16X1 = 1,
  DFT3D_PREC_FP16X1 = 2,
  DFT3D_PREC_BF16X6 = 3,
  DFT3D_PREC_BF16X9 = 4,
  DFT3D_PREC_FP16X3 = 5
};

/* Status codes. */
enum dft3d_status {
  DFT3D_OK = 0,
  DFT3D_ERR_INVALID_ARG = -1,          /* null pointer, bad enum, bad sign */
  DFT3D_ERR_UNSUPPORTED_SIZE = -2,     /* n_d outside [1, 4096] */
  DFT3D_ERR_UNSUPPORTED_SCHEDULE = -3, /* schedule/layout/precision combination */
  DFT3D_ERR_NO_DEVICE = -4,            /* no HIP device visible */
  DFT3D_ERR_OUT_OF_MEMORY = -5,        /* device allocation failed */
  DFT3D_ERR_HIP = -6,                  /* a HIP runtime call failed */
  DFT3D_ERR_WORKSPACE_TOO_SMALL = -7   /* dft3d_set_workspace buffer too small */
};

/* Option keys for dft3d_plan_set_option / dft3d_plan_get_option.  Setting
 * an option rebuilds the pass list (host work plus a table upload). */
enum dft3d_option {
  DFT3D_OPT_PRECISION = 1,   /* enum dft3d_precision; default FP32 */
  DFT3D_OPT_TILE = 2,        /* pencils per workgroup, power of two; 0 = default */
  DFT3D_OPT_XCD_REMAP = 3,   /* 1 = map consecutive tiles to one XCD; default 1 */
  DFT3D_OPT_SPLIT_MAX = 4,   /* longest axis done in one pass; longer axes
                                are split four-step; 0 = default */
  DFT3D_OPT_NONTEMPORAL = 5, /* streaming (non-temporal) loads and stores:
                                0 off, 1 on, 2 automatic (default): on with
                                the persistent kernels for arrays of 256 MiB
                                or more, off otherwise */
  DFT3D_OPT_PERSISTENT = 6,  /* 1 = persistent prefetching pass kernels
                                where compiled (default 1) */
  DFT3D_OPT_SLAB_GROUP = 7,  /* slab: planes per row/column group, 0 = all
                                planes, -1 = automatic (default) */
  DFT3D_OPT_FUSED_PLANE = 8, /* slab, FP32: 1 = 2D DFT of each (n1, n2)
                                plane in one pass when n1, n2 are in
                                [16, 128] (the plane stays in LDS between
                                rows and columns); default 1 */
  DFT3D_OPT_FUSED_AXES = 9,  /* volumetric, FP32: 1 = the second half of
                                one axis and the first half of the next in
                                one pass where the split factors match
                                (a_d = b_{d-1} = 16 or 32: 256^3, 1024^3),
                                in the natural layout and in the shuffled
                                one, whose inverse runs the forward's
                                passes transposed (second half of an axis
                                with the first half of the next inner
                                axis, Section 2.4); default 1 */
  DFT3D_OPT_PENCIL_GROUP = 10, /* pencil, FP32, powers of two: planes of
                                axis 0 per group of the first two passes
                                (rounded down to a power of two), so a
                                group's intermediate can stay in the
                                Infinity Cache; 0 = all planes at once
                                (default), -1 = groups of up to 256 MB for
                                arrays of 256 MiB or more where the
                                one-sided streaming kernels exist (length
                                1024); slower than 0 at 1024^3 as measured,
                                offered to the autotuner */
  DFT3D_OPT_BATCH_LAUNCH = 11, /* batched calls (Section 4's point that no
                                one decomposition suits every shape, served
                                by one pool of workers): 0 = one launch per
                                pass level (default); 1 = one persistent
                                launch for the whole batch, replayed from a
                                HIP graph the library builds, used when every
                                plan of the batch has 1 */
  DFT3D_OPT_MOVE_ONLY = 12,  /* the data movement of a schedule alone, for
                                the time breakdown the paper draws for its
                                decompositions (Section 4.3: communication,
                                packing and local DFTs): 0 = off (default);
                                1 = every pass keeps its loads, LDS
                                exchanges and stores with the radix stages
                                (butterflies and twiddles) removed, so the
                                output is a fixed permutation of the input;
                                2 = every pass is a plain copy of the array
                                (output = input), the HBM floor.  FP32,
                                NATURAL layout, powers of two; fused plane,
                                fused axes and grouped pencil passes are
                                turned off (their unfused passes run);
                                otherwise UNSUPPORTED_SCHEDULE */
  DFT3D_OPT_MFMA_LEAF = 13,  /* split-precision passes: the length of the
                                DFT leaves on the matrix cores (Section 2.1,
                                eqs. (1)-(2): the small DFT as a dense
                                product): 16 or 32; 0 = the default for
                                each pass length and precision (32 for
                                lengths 128, 256, 4096 and for fp16 forms at
                                1024, else 16).  Leaves of 32 exist for
                                lengths 32^s r with r < 16 (32 .. 256,
                                1024 .. 4096); other lengths keep leaves of
                                16.  Other values: INVALID_ARG */
  DFT3D_OPT_RADICES = 14,    /* the radix sequence of the passes of one
                                length (Section 2.2: the 1D DFT as stages of
                                smaller DFTs, eq. (3)): the stage radices, 8
                                bits each, first stage in the lowest byte,
                                each one of 2, 3, 4, 5, 7, 8, 10, 11, 13, 16,
                                at most 8 stages, product n <= 2048 (the
                                composites 10 and 16 only below 2048, not
                                with 11 or 13).  FP32
                                passes of length n without a four-step
                                twiddle then run the mixed-radix kernel
                                with these stages (powers of two too); other
                                lengths keep their default.  0 = default
                                (the compiled sequence of each length).
                                Workgroup size is set by DFT3D_OPT_TILE:
                                pencils per workgroup times the kernel's
                                threads per pencil.  Other values:
                                INVALID_ARG */
  DFT3D_OPT_RADER = 15,      /* prime lengths n whose n - 1 has no prime
                                factor above 13: Rader's identity, the DFT
                                as a cyclic convolution of length n - 1
                                done with two mixed-radix FFTs of that
                                length, instead of Bluestein (two FFTs of
                                the power of two >= 2n - 1).  1 (default) =
                                Rader for the primes a kernel is compiled
                                for, 2 = for every such prime (a generic
                                kernel for the others, measured slower than
                                Bluestein), 0 = Bluestein.  Other values:
                                INVALID_ARG */
  DFT3D_OPT_HALVES = 16,     /* FP32 passes as two half-length transforms
                                after a radix-2 split (the four-step
                                factorisation of eq. (3) with radix 2
                                first), in tiles of twice the pencils, so
                                that the strided row segments are longer:
                                the pencil schedule's rotate-on-write passes
                                of length 2048 (16 pencils, 128-byte
                                segments) and the slab schedule's strided
                                passes of lengths 1024 (32 pencils, 256
                                bytes) and 2048 (16).  1 (default) = on,
                                0 = the whole-length kernels.  Taken when
                                DFT3D_OPT_TILE is 0 or the halves kernel's
                                tile.  Other values: INVALID_ARG */
  DFT3D_OPT_PENCIL_ORDER = 17, /* pencil schedule, every axis a power of two
                                and unsplit: the intermediate orders, all
                                ending in the natural order.  0 = each pass
                                writes its axis slowest (the rotation
                                xyz -> yzx of eq. (8)); 1 = the first pass
                                swaps the two fastest axes and the second
                                writes (C, B, A); 2 = (A, B, C) ->
                                (B, C, A) -> (C, A, B) -> (A, B, C), every
                                pass loading pencils one plane apart and
                                storing rows one row length apart; -1
                                (default) = 2 for split precision and for
                                arrays with an axis of 2048, else 0 (the
                                faster order measured for each).  Other
                                values: INVALID_ARG */
  DFT3D_OPT_NUM_PASSES = 100 /* read-only: number of kernel launches */
};

/* Text for a status code; never NULL. */
const char* dft3d_status_string(int status);

/* Build a plan for a (n0, n1, n2) complex64 transform: the 3D DFT of Section
 * 2.1 eqs. (1)-(2) applied along the three axes (Section 2.3), decomposed as
 * the schedule says (slab: eq. (6), Fig. 5; pencil: eq. (8), Fig. 6;
 * volumetric: Fig. 9, eqs. (13)-(17)).  As in the paper's Fig. 10, the shape
 * and layout are described once and the transform is run many times.  Each
 * n_d is in
 * [1, 4096].  Powers of two run on every schedule.  Other lengths (the
 * paper's experiments use powers of two; it leaves sizes its process grid
 * does not divide to future work, Section 3.2) run with FP32 precision and
 * the natural layout on every schedule (AUTO picks pencil), one pass per
 * such axis (rotate-on-write in the pencil schedule, in layout in the slab
 * and volumetric schedules): a mixed-radix pass (radices 2, 3, 4, 5, 7, 8,
 * 10, 11, 13, 16) when every prime factor of n_d is at most 13, else for
 * the primes n_d whose n_d - 1 has that property and that a Rader kernel is
 * compiled for a Rader pass (a circular convolution of length n_d - 1 done
 * with two mixed-radix FFTs, see DFT3D_OPT_RADER), else a Bluestein pass (the DFT of length n as a circular
 * convolution of length m, the power of two >= 2n - 1, up to 8192, done
 * with two power-of-two FFTs in the same workgroup).  Split precisions, the shuffled layout and
 * move-only plans with such lengths return UNSUPPORTED_SCHEDULE.  The
 * workspace is N * 8 bytes as for powers of two.  Validates the arguments
 * first
 * (INVALID_ARG / UNSUPPORTED_SIZE / UNSUPPORTED_SCHEDULE), then needs a HIP
 * device (NO_DEVICE), then allocates and uploads the twiddle tables on the
 * current device (OUT_OF_MEMORY / HIP_ERROR).  *out receives the handle, or
 * NULL on error.  The workspace is not allocated here. */
int dft3d_plan(int64_t n0, int64_t n1, int64_t n2, int schedule, int layout,
               dft3d_plan_t* out);

/* Describe the pass list a plan with the given options would use (the
 * sequence of batched local DFTs and redistributions of Section 2.4 that the
 * schedule becomes on one device), without
 * touching any device: keys[i] / values[i] (nopts pairs, as for
 * dft3d_plan_set_option; both may be NULL when nopts == 0) are applied to the
 * default options, then a NUL-terminated JSON text is written into buf (at
 * most len bytes, truncated if needed) and the full length is stored in
 * *needed (may be NULL).  Same argument validation as dft3d_plan. */
int dft3d_plan_describe(int64_t n0, int64_t n1, int64_t n2, int schedule,
                        int layout, const int* keys, const int64_t* values,
                        int nopts, char* buf, size_t len, size_t* needed);

/* Set / read one option of a plan (enum dft3d_option): the tuning choices
 * of a decomposition that do not change the result in exact arithmetic (the
 * four-step split of a long axis, Section 3.2; tile shapes; the leaf
 * arithmetic of the split-precision forms).  set_option validates the value
 * (INVALID_ARG), rebuilds the pass list and uploads its tables; on failure
 * (OUT_OF_MEMORY / HIP_ERROR) the previous pass list and options stay in
 * force.  get_option writes the current value to *value.  NULL plan or value:
 * INVALID_ARG. */
int dft3d_plan_set_option(dft3d_plan_t plan, int key, int64_t value);
int dft3d_plan_get_option(dft3d_plan_t plan, int key, int64_t* value);

/* Bytes of device workspace dft3d_execute needs (0 if none): the second
 * buffer a redistribution writes into when it cannot work in place (the
 * target B of eq. (12)); N * 8 bytes for the pencil and volumetric
 * schedules, 0 for slab.  NULL arguments: INVALID_ARG. */
int dft3d_workspace_size(dft3d_plan_t plan, size_t* bytes);

/* Hand the plan a caller-owned device buffer of `bytes` bytes to use as
 * workspace (WORKSPACE_TOO_SMALL if below dft3d_workspace_size).  The plan
 * does not free it.  Without this call the plan allocates its own on the
 * first execute and frees it in dft3d_destroy.  Passing NULL reverts to
 * plan-owned workspace. */
int dft3d_set_workspace(dft3d_plan_t plan, void* dev_ptr, size_t bytes);

/* Enqueue the transform on `stream` (a hipStream_t; NULL = default stream)
 * and return: the passes of the plan's schedule, each a batched 1D DFT
 * (Section 2.1, eq. (3) inside a pass) with the redistribution to the next
 * axis folded into its loads and stores (Section 2.3 eqs. (6)-(8); Section
 * 3.2, Fig. 9 and eqs. (13)-(17) for the volumetric schedule).  in, out: device pointers of n0 n1 n2 complex64, distinct and
 * non-overlapping (in == out is INVALID_ARG); in is never written.
 * sign = -1 forward, +1 inverse, anything else INVALID_ARG.  The current
 * device must be the one the plan was created on (INVALID_ARG otherwise).
 * Launch errors are returned (HIP_ERROR); faults inside kernels surface at
 * the caller's next synchronisation.  Once the plan has a workspace (bound with
 * dft3d_set_workspace or allocated by an earlier execute) and has executed
 * once on the device, a call only launches kernels on `stream`: no
 * allocation, synchronisation or memset, so it may be captured into a HIP
 * graph and replayed (the graph keeps the buffer pointers it was captured
 * with). */
int dft3d_execute(dft3d_plan_t plan, const void* in, void* out, int sign,
                  void* stream);

/* Enqueue `count` transforms of possibly different shapes together (the
 * paper finds that no single decomposition is fastest for every size,
 * Section 4; one pool of workers serves every problem, as its threads serve
 * both computation and packing in Fig. 11): one kernel launch per pass level
 * covers the tiles of every problem at that level, or, with
 * DFT3D_OPT_BATCH_LAUNCH = 1 on every plan, one persistent launch runs every
 * level (a device ticket queue; a tile of pass k of a problem starts after
 * every tile of its pass k - 1; the launch is replayed from a HIP graph the
 * library builds once per descriptor set).
 *
 * plans[i] describes problem i (the same plan may appear more than once),
 * in[i] and out[i] are its device buffers (same rules as dft3d_execute;
 * distinct problems must not share buffers).  Problems whose workspaces
 * would be shared (a repeated plan, or distinct plans bound to overlapping
 * buffers with dft3d_set_workspace) get private workspaces for the batched
 * call, since their passes run at the same time.  The first call for a given
 * sequence of plans builds the work descriptors; later calls with the same
 * sequence only refresh the buffer pointers.  Plans whose passes exceed
 * length 256 or are split four-step (volumetric) run one after another.
 * count == 0 is a no-op.  Plans must use the NATURAL layout and FP32
 * (UNSUPPORTED_SCHEDULE otherwise).  Not thread-safe for concurrent calls
 * with overlapping plans; calls with the same plans must be ordered (the
 * persistent form's counters belong to its descriptor set).  A call with the
 * same plans, buffers and sign as the previous one reuses the descriptors
 * already on the device (no upload).  The persistent form's waits are
 * bounded: with DFT3D_BATCH_CHECK=1 in the environment a call waits for its
 * launch and returns DFT3D_ERR_HIP if a wait ran out (never expected).
 * Capture into a HIP graph: on a capturing stream the call records only its
 * kernel launches, so an earlier call outside the capture must have used
 * exactly these plans, buffers and sign (and bound every workspace);
 * otherwise it returns DFT3D_ERR_UNSUPPORTED_SCHEDULE before enqueueing
 * anything.  Those descriptors then stay fixed while the plans live (later
 * calls with other buffers get descriptor sets of their own); destroying or
 * changing a plan invalidates graphs that captured it. */
int dft3d_execute_batched(const dft3d_plan_t* plans, const void* const* in,
                          void* const* out, int count, int sign, void* stream);

/* Describe, without touching any device, how dft3d_execute_batched lays out
 * `count` problems of shapes shapes[3i .. 3i+2] planned with `schedule`
 * (NATURAL layout, default options) when `launch` is the
 * DFT3D_OPT_BATCH_LAUNCH value of every plan: a NUL-terminated JSON text with
 * the work items in level-major order (problem, pass, first tile, tiles,
 * the item it waits for, transform length, plane rows, pencils, pencils per
 * tile), the per-level launches, the ticket total and the workgroup shape.
 * Written into buf (at most len bytes, truncated if needed); the full length
 * goes to *needed (may be NULL).  Same argument validation as dft3d_plan. */
int dft3d_batch_describe(const int64_t* shapes, int count, int schedule, int launch,
                         char* buf, size_t len, size_t* needed);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as dft3d_execute on the same plan (same kernels, bitwise equal
 * output), with the workspace taken from a static device array of
 * DFT3D_NOALLOC_MAX_WORKSPACE bytes that the library holds on every GPU it
 * runs on until the process ends, instead of a plan-owned or bound buffer.
 * Never allocates or frees device memory and ignores any workspace bound to
 * the plan.  in, out, sign, stream and the device rule are as for
 * dft3d_execute.  A plan whose dft3d_workspace_size exceeds the maximum
 * (transforms above 2^24 points on the PENCIL and VOLUMETRIC schedules) is
 * rejected with DFT3D_ERR_WORKSPACE_TOO_SMALL before anything is enqueued;
 * SLAB plans need no workspace and take any size.  All calls on one GPU share
 * that GPU's array: calls whose execution may overlap in time on one GPU
 * (different streams without ordering, different host threads) race and give
 * wrong results; calls in one stream's order are safe.  The first call on a
 * device looks the array's address up (no allocation). */
#define DFT3D_NOALLOC_MAX_WORKSPACE ((size_t)128 << 20)
int dft3d_execute_noalloc(dft3d_plan_t plan, const void* in, void* out, int sign,
                          void* stream);

/* Autotuner (the choice of decomposition per problem size that Section 4
 * measures by hand): time candidate schedules and kernel options (pencil with and
 * without the persistent kernels, split long axes, other tiles, grouped
 * first passes, other radix sequences for axis lengths that are not powers
 * of two; slab; volumetric) for a (n0, n1, n2) transform on the
 * current device, on `in`
 * and `out` (device buffers of n0 n1 n2 complex64; out is overwritten), in
 * stream order on `stream`, and record the fastest: DFT3D_SCHED_AUTO plans
 * of that shape created afterwards use it (their precision is kept).  The
 * choice is kept for the process and, when the environment variable
 * DFT3D_TUNE_CACHE names a file, written there and read back by later
 * processes on the same GPU architecture.  Candidates allocate their own
 * workspace.  best_schedule and best_ms (may be NULL) receive the choice and
 * its forward time.  Blocks until the timing is done. */
int dft3d_autotune(int64_t n0, int64_t n1, int64_t n2, const void* in,
                   void* out, void* stream, int* best_schedule,
                   double* best_ms);

/* Release the plan, its device tables, any plan-owned workspace and the
 * batched descriptor sets that use it (waiting for their last launch).
 * NULL is accepted (DFT3D_OK). */
int dft3d_destroy(dft3d_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* DFT3D_H */
