/*
 * sosfilt.h -- C ABI of the MI355X (gfx950) cascaded-biquad filter library.
 *
 * The library filters long signals through a cascade of K second-order
 * sections (Section II, eq. general_cascaded_equation and eq.
 * complex_second_order):
 *
 *   y_k[n] = b0 x_k[n] + b1 x_k[n-1] + b2 x_k[n-2] - a1 y_k[n-1] - a2 y_k[n-2],
 *   x_1 = x,  x_k = y_{k-1},  y = y_K,  zero initial state.
 *
 * Each group of N*L samples is taken in the stride-N layout of Section V:
 * lane l of a group of L lanes holds x[m + l N] for block m.  With L = 16 (a
 * DPP row, the default) a 64-wide wavefront carries four such groups from
 * four different tiles; with L = 32 two, with L = 64 one.
 * This turns each group into the block-tridiagonal system of eq.
 * multi_block_A.  That
 * system is solved per section by the PH factorisation (Section VI-B) or by
 * cyclic reduction (Section VI-C); the permuted layout is kept across all K
 * sections (Section VII-B), so one permutation and one de-permutation serve
 * the whole cascade.  Groups inside a tile are chained by the per-section
 * boundary values (x[-2], x[-1], y[-2], y[-1]) as in Section V; tiles are
 * chained by the cascade's 2K-dimensional state (see sos_plan_info).
 *
 * Conventions for every entry point:
 *  - "host" pointers are CPU memory; "device" pointers are GPU memory on the
 *    device current when the call is made.  All arrays are contiguous.
 *  - Calls never throw; they return a sos_status.  Arguments are checked
 *    before anything is enqueued: on any error nothing is launched and no
 *    output is written.
 *  - Filtering calls are asynchronous on the given HIP stream (NULL = the
 *    legacy default stream), do not allocate and do not synchronise.
 *  - A plan is immutable once created and may be used from several threads
 *    and streams at once; it must outlive all work enqueued with it.
 */
#ifndef SOSFILT_H
#define SOSFILT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sos_plan_s *sos_plan_t;      /* opaque, owned by the caller */
typedef struct ihipStream_t *sos_stream_t;  /* a hipStream_t */

typedef enum {
    SOS_OK = 0,
    SOS_E_ARG = 1,          /* null/invalid pointer, size, aliasing, bad enum */
    SOS_E_COEF = 2,         /* a0 == 0 or a non-finite coefficient */
    SOS_E_UNSTABLE = 3,     /* a section with |a2| >= 1 or |a1| >= 1 + a2 (after a0 division) */
    SOS_E_UNSUPPORTED = 4,  /* N, L, dtype combination or K not built */
    SOS_E_DEVICE = 5,       /* a HIP call failed (no device, launch error) */
    SOS_E_NOMEM = 6,        /* host or device allocation failed (plan creation only) */
    SOS_E_SCRATCH = 7       /* sos_filt_static: the call needs more workspace than the
                               library's static buffer holds (SOS_STATIC_SCRATCH_BYTES) */
} sos_status;

typedef enum {
    SOS_F32 = 0,
    SOS_F64 = 1,
    SOS_F16 = 2,   /* product type of SOS_BLOCK only: FP16 MFMA, FP32 accumulation */
    SOS_BF16 = 3   /* product type of SOS_BLOCK only: BF16 MFMA, FP32 accumulation */
} sos_dtype;

typedef enum {
    SOS_AUTO = 0,        /* PH for every section (the faster of PH and CR on MI355X at
                            every N, and free of the CR guard); where the lane runs
                            live in the workspace (N = 256 .. 1024, and N = 128 with
                            FP64 I/O) and K <= 16, SOS_PH_DEFERRED, which passes
                            the runs once for all sections (4-5 times faster there) */
    SOS_PH = 1,          /* PH factorisation (Section VI-B) for every section */
    SOS_CR = 2,          /* cyclic reduction (Section VI-C), guard still applies */
    SOS_PH_DEFERRED = 3, /* PH with the homogeneous correction (eq. PH_forward) of all
                            sections deferred to the end of the cascade and applied as
                            one FP64 matrix-core product; FP64 arithmetic, N >= 16
                            (up to 1024, L = 16), K <= 16 */
    SOS_SCALAR = 4,      /* comparison point: scalar filtering (the plain recurrence of
                            Section II, one lane per segment, run-in carry); K <= 16,
                            N ignored */
    SOS_BLOCK = 5        /* block filtering (Section IV, eq. block_filtering_equation):
                            the 16 x 16 Toeplitz product H x on MFMA in the
                            compute_dtype (SOS_F64, SOS_F16 or SOS_BF16; FP32
                            accumulation for the latter two, with error-free operand
                            slices, see SOS_FLAG_SLICES), the boundary terms, the
                            block-to-block recurrence and the carries in FP64;
                            K <= 32, N ignored */
} sos_solver;

/* Plan flags. */
#define SOS_FLAG_HOST_ONLY 0x1u   /* build the FP64 host tables only; the plan
                                     can be queried but not used to filter */
#define SOS_FLAG_CARRY_SCAN 0x2u  /* carry between tiles by the exact scan
                                     whenever the plan supports it (see
                                     sos_workspace_size) */
#define SOS_FLAG_CARRY_RUNIN 0x4u /* always carry by the run-in (not with
                                     SOS_FLAG_CARRY_SCAN) */
#define SOS_FLAG_ADJ_SAVE 0x8u    /* adjoint: keep every section's output (see
                                     sos_backward_workspace_size) */
#define SOS_FLAG_ADJ_RECOMPUTE 0x10u /* adjoint: checkpoint the cascade state
                                     per group and recompute section inputs
                                     (not with SOS_FLAG_ADJ_SAVE) */
/* SOS_BLOCK with compute_dtype SOS_F16 or SOS_BF16: slices per operand of
 * the Toeplitz products, 1..4 (0 = the default, 3 for FP16 and 4 for BF16).
 * 1 rounds both operands once to the product type.  S >= 2 cuts both into S
 * integer slices of W bits (W = 10 for FP16, 8 for BF16) after a
 * power-of-two scale per 16-sample block (Ozaki et al., 2012): the matrix
 * cores then accumulate every order of slice products exactly in FP32, and
 * the product's error is that of the slices cut off, about 2^(-W (S-1)) of
 * the block's largest value.  Orders a + b < S are formed: S (S + 1) / 2
 * slice products per section and group of 256 samples. */
#define SOS_FLAG_SLICES(s) (((uint32_t)(s) & 7u) << 8)
#define SOS_FLAG_SLICES_MASK 0x700u

typedef struct {
    int32_t io_dtype;       /* sos_dtype of x and y (default SOS_F32) */
    int32_t compute_dtype;  /* sos_dtype of the in-kernel arithmetic (default SOS_F64); SOS_F16
                               and SOS_BF16 only with SOS_BLOCK */
    int32_t solver;         /* sos_solver (default SOS_AUTO) */
    int32_t N;              /* blocks per group: 8, 16, 32 or 64 (0 = 32); also 4 for single
                               signals with SOS_AUTO, SOS_PH or SOS_CR and L = 16; and 128, 256,
                               512 and 1024 for single signals with SOS_AUTO, SOS_PH, SOS_CR or
                               SOS_PH_DEFERRED, FP64 arithmetic and L = 16.  At N = 128 with
                               FP32 I/O a lane's run (128 doubles) stays in registers for PH
                               and CR, one wavefront per SIMD; the other wide runs do not fit
                               on chip and live in the workspace (sos_workspace_size) */
    int32_t L;              /* samples per block = lanes per group: 16 (a DPP row), 32 or 64
                               (the whole wavefront); 32 and 64 with SOS_AUTO, SOS_PH and
                               SOS_CR only (0 = 16) */
    int32_t tile_groups;    /* groups per tile (0 = chosen per call from n) */
    uint32_t flags;         /* SOS_FLAG_* */
} sos_opts;

/* Limits. */
#define SOS_MAX_SECTIONS 64

/*
 * sos_plan -- validate coefficients and build the per-section tables.
 *
 * sos   host, [K][6] row-major float64, rows (b0, b1, b2, a0, a1, a2) as in
 *       eq. complex_second_order with the denominator a0 + a1 z^-1 + a2 z^-2.
 *       Each row is divided by its a0 (a0 = 0 -> SOS_E_COEF).  If every b0 is
 *       nonzero and the running products of 1/b0 stay within range, b0 is
 *       factored out as in eq. simple_second_order and the product of the b0
 *       is applied once at the store.  Copied; the caller may free it.
 * K     1..SOS_MAX_SECTIONS.
 * opts  host, may be NULL for the defaults.
 * out   host, receives the plan handle (unchanged on error).
 *
 * Tables (FP64 on the host, converted to the compute dtype on the device):
 * u_{1,m}, u_{2,m} (Section VI-A), the matrix C of eq. C and the powers of
 * -C used by the terminal-block scan (Section VI-B), the cyclic-reduction
 * coefficients of eq. cr_coeff_update per level (f/e, e, c, d) and the
 * terminal-block coefficients of eq. cr_terminal_block, and the cascade's
 * one-step state transition (2K x 2K).  The cyclic-reduction guard runs
 * here: a level whose r^(2^i) < 2^-60 is flushed to zero coupling; a section
 * with any |f/e|, |c| or |d| above 64 at a remaining level is solved with PH
 * (reported by sos_plan_query).  No division happens on the device.
 */
sos_status sos_plan(const double *sos, int32_t K, const sos_opts *opts, sos_plan_t *out);

/* Release the plan and its device tables.  NULL is accepted. */
sos_status sos_plan_destroy(sos_plan_t plan);

typedef struct {
    int32_t K, N, L;
    int32_t io_dtype, compute_dtype;
    int32_t b0_factored;        /* 1 if the b0 of every section was factored out */
    int64_t warm_samples;       /* W: samples of run-in after which the state transition's
                                   infinity norm is below 2^-64 (FP64 I/O and arithmetic)
                                   or 2^-40 (otherwise: 2^16 below FP32's unit roundoff);
                                   a multiple of N*L */
    double gain;                /* product of the b0 applied at the store (1 if not factored) */
    double transition_norm_W;   /* infinity norm of the cascade state transition over W samples */
    int32_t simds;              /* SIMDs of the plan's device (0 for a host-only plan) */
    int32_t waves_per_simd;     /* resident wavefronts per SIMD of the plan's kernel (0: host-only) */
    int32_t block_slices;       /* SOS_BLOCK: slices per operand of the products (1 otherwise) */
    int32_t reserved;           /* 0 */
} sos_plan_info;

/* info        host, filled in.
 * solver      host [K] or NULL: per section SOS_PH or SOS_CR as run. */
sos_status sos_plan_query(sos_plan_t plan, sos_plan_info *info, int32_t *solver);

/* Samples per tile that sos_filt's run-in carry uses for n samples: the
 * plan's tile_groups, or the launch-shape model: the shortest tile that
 * gives every SIMD at most m wavefronts (four tiles each), m the largest
 * power of two of resident wavefronts per SIMD for the plan's kernel.  The
 * exact carry (see sos_workspace_size) uses the same model with no run-in. */
int64_t sos_plan_tile(sos_plan_t plan, int64_t n);

/* Host FP64 tables, for inspection and tests.  Copies min(count, size) values
 * into out (host) and returns the table's size in *size (host, may be NULL).
 * section is ignored for SOS_TABLE_TRANSITION and SOS_TABLE_THETA; the
 * SOS_PH_DEFERRED tables exist only for plans with that solver. */
typedef enum {
    SOS_TABLE_ROWS = 0,        /* 5: b0 b1 b2 a1 a2 as the kernel uses them */
    SOS_TABLE_U1 = 1,          /* N: u_{1,m} */
    SOS_TABLE_U2 = 2,          /* N: u_{2,m} */
    SOS_TABLE_C = 3,           /* 4: e g f d (eq. C), row-major */
    SOS_TABLE_PH_POWERS = 4,   /* 4 log2 L = 16: (-C)^(2^j), row-major, j = 0..3 */
    SOS_TABLE_CR_LEVELS = 5,   /* 4 log2 N: per level f/e, e, c, d */
    SOS_TABLE_CR_TERMINAL = 6, /* 2: e, f of eq. cr_terminal_block */
    SOS_TABLE_CR_POWERS = 7,   /* 4 log2 L = 16: T^(2^j), T = [[0, 1], [-f, -e]] */
    SOS_TABLE_TRANSITION = 8,  /* (2K)^2: one-step cascade state transition, row-major */
    SOS_TABLE_THETA = 9,       /* N x 2K: SOS_PH_DEFERRED correction matrix, row-major
                                  (response of the last section at block m to a unit entry
                                  state component (y_j[-2], y_j[-1])); section ignored */
    SOS_TABLE_COUPLING = 10    /* 4k: for section k, the 2x2 blocks (j = 0..k-1) giving its
                                  terminal values from section j's entry state */
} sos_table;

sos_status sos_plan_table(sos_plan_t plan, int32_t table, int32_t section,
                          double *out, int32_t count, int32_t *size);

/*
 * Device workspace bytes sos_filt uses for n samples.  For N = 256 .. 1024,
 * and N = 128 with FP64 I/O or SOS_PH_DEFERRED: the lane runs of every
 * wavefront of the launch (N x 64 doubles per wavefront, at most one
 * wavefront per SIMD; PH and CR, which pass the runs once per section, also
 * at most 256 MB in all, the last-level cache of MI355X: 512 wavefronts at
 * N = 1024), required.  N = 128 with FP32 I/O and PH or CR needs none.
 * Otherwise
 * 0 when it carries the state between tiles by the run-in, else the size
 * of the exact carry's buffers.  The exact carry (FP64 arithmetic, solvers AUTO, PH or CR,
 * K <= 16, L = 16, N = 8 .. 64) runs every tile twice, once from zero section states to get its
 * end state c_t and once from the scanned true state, with a log-depth scan
 * S_t = c_t + Phi^T S_{t-1} in between (Phi the cascade's one-step state
 * transition).  sos_filt takes it when the run-in would be longer than 1.2
 * tiles (a signal short against its run-in, poles near the unit circle) and
 * the run-in it saves, K (W - tile) section-samples, is at least 8192 (below
 * that the scan's extra launches cost more), or always with
 * SOS_FLAG_CARRY_SCAN; never with SOS_FLAG_CARRY_RUNIN.
 */
size_t sos_workspace_size(sos_plan_t plan, int64_t n);

/*
 * sos_filt -- y = cascade(x), zero initial state.
 *
 * x, y       device, n samples of the plan's io_dtype; must not overlap
 *            (SOS_E_ARG): tiles re-read input that precedes them.
 * n          >= 0; n == 0 is a no-op.  Any n is accepted: the last group is
 *            zero-padded and only n outputs are written.
 * workspace  device, at least sos_workspace_size(plan, n) bytes, 16-byte
 *            aligned, contents on entry irrelevant; may be NULL, which keeps
 *            the run-in carry (SOS_E_ARG if the size is not 0 and the plan
 *            has SOS_FLAG_CARRY_SCAN or N > 64).
 * stream     HIP stream the kernels are enqueued on.
 * No allocation and no synchronisation in either carry.
 */
sos_status sos_filt(sos_plan_t plan, const void *x, void *y, int64_t n,
                    void *workspace, sos_stream_t stream);

/*
 * sos_filt_static -- sos_filt for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result as sos_filt(plan, x, y, n, ws, stream) with a
 * workspace of sos_workspace_size(plan, n) bytes, but the workspace is a
 * fixed buffer of SOS_STATIC_SCRATCH_BYTES inside the library's device code,
 * one per GPU, held from the first call on that GPU until the process ends.
 *
 * x, y, n, stream  as sos_filt (device x and y on the current device, which
 *                  must be the plan's).
 * Returns SOS_E_SCRATCH, enqueuing nothing, when sos_workspace_size(plan, n)
 * exceeds SOS_STATIC_SCRATCH_BYTES (only the exact carry and the lane runs
 * of wide groups use a workspace; other calls need none).  The first call on a device
 * looks up the buffer's address there (SOS_E_DEVICE if that fails).  No
 * allocation, no synchronisation.  Every call on one GPU uses the same
 * buffer, whatever the plan or stream: calls whose launches can overlap on
 * one GPU (different streams, or different host threads without ordering)
 * race on it and must be serialised by the caller.  The buffer keeps the
 * last call's contents; the kernels write every word they read first.
 */
#define SOS_STATIC_SCRATCH_BYTES (16u << 20)

sos_status sos_filt_static(sos_plan_t plan, const void *x, void *y, int64_t n, sos_stream_t stream);

/*
 * Batched ragged channels (one launch for many independent signals, each
 * with its own cascade).  The per-channel work is exactly sos_filt's: the
 * same tile kernels (Sections V to VII) run on every channel, and only the
 * scheduling is shared: each channel is cut into tiles, four tiles form one
 * wavefront's work item, and the items of all channels are launched
 * together, costliest first.
 *
 * sos_batch_plan -- fix the channel set and lengths once (allocates).
 *
 * plans    host [C]: channel c is filtered with plans[c] (the same plan may
 *          serve several channels).  All plans must share N (8 .. 64; the
 *          narrow and wide widths are single-signal only), L, io_dtype and
 *          compute_dtype (else SOS_E_UNSUPPORTED), and either all use
 *          SOS_AUTO, SOS_PH or SOS_CR, or all use SOS_BLOCK (block filtering,
 *          one workgroup per four tiles of a channel, with that channel's
 *          Toeplitz operands in LDS; its groups are 256 samples whatever
 *          N).  SOS_PH_DEFERRED and SOS_SCALAR give SOS_E_UNSUPPORTED.  The
 *          plans must outlive the batch: the batch refers to their device
 *          tables.  sos_batch_replan keeps the batch's kind (block or not).
 * C        number of channels, >= 1.
 * n        host [C]: channel lengths, >= 0.
 * offsets  host [C] or NULL: first sample of channel c in the concatenated
 *          x and y buffers.  NULL packs the channels densely in order
 *          (offset[c] = n[0] + ... + n[c-1]).  Channels must not overlap.
 *          Any offset is accepted at full speed: a channel starting off
 *          a 16-byte boundary is filtered over a span that begins up to
 *          three samples (FP64: one) earlier, read as zeros and never
 *          stored, so that its groups move as 16-byte vectors.
 * opts     host, may be NULL: tile_groups > 0 caps the groups per tile
 *          (0 = chosen by a makespan model over candidate caps from every
 *          channel's length, run-in and K, and the kernel's residency);
 *          flags SOS_FLAG_HOST_ONLY
 *          builds the schedule without device memory (queries only, and
 *          host-only plans are then accepted); max_channels, max_samples
 *          and max_sections reserve room for later sos_batch_replan calls
 *          of up to that many channels, samples in all, and sections per
 *          channel (0 = this set's size).
 * out      host, receives the batch handle (unchanged on error).
 *
 * Everything a sos_filt_batched launch depends on is fixed here: its grid
 * (the most work items the reserved room allows), its LDS (the reserved
 * sections) and its kernel instance.  A batch created with any of the three
 * reservations above runs the kernel instance that serves every channel
 * (sections of both solvers, b0 kept in the numerator); without one, the
 * instance of this channel set.  So a sos_filt_batched launch captured in a
 * HIP graph replays correctly after any number of sos_batch_replan calls:
 * the kernel reads the current channel set and item count from the batch's
 * device descriptors.
 */
typedef struct sos_batch_s *sos_batch_t;   /* opaque, owned by the caller */

typedef struct {
    int32_t tile_groups;
    uint32_t flags;
    int32_t max_channels;
    int32_t max_sections;  /* room for replans: largest K of a later channel set
                              (0 = this set's largest K) */
    int64_t max_samples;
} sos_batch_opts;

sos_status sos_batch_plan(const sos_plan_t *plans, int32_t C, const int64_t *n,
                          const int64_t *offsets, const sos_batch_opts *opts, sos_batch_t *out);

/* Release the batch and its device schedule.  NULL is accepted. */
sos_status sos_batch_destroy(sos_batch_t batch);

/*
 * sos_batch_replan -- give an existing batch a new channel set (a serving
 * loop's next request) without allocating: the schedule is rebuilt on the
 * host and copied, asynchronously on `stream`, into the batch's device
 * descriptors through its pinned staging buffer.  Arguments as for
 * sos_batch_plan; the plans must share the batch's N, io_dtype,
 * compute_dtype and slices, and (for a batch created without a
 * reservation) fit its kernel instance: no unfactored b0 where the batch's
 * channels all had it factored, and the same solver class unless the batch
 * mixed classes (SOS_E_UNSUPPORTED).  SOS_E_NOMEM if the new schedule does
 * not fit the room fixed at creation (channels, work items, sections,
 * adjoint items and rows); on any error the batch keeps its previous
 * channel set.  Later launches with the batch must be on `stream` (or
 * ordered after it).  The call waits only for the previous replan's copy,
 * so it never waits for a kernel.  sos_filt_batched launches captured
 * before the replan stay valid (see sos_batch_plan); captured launches of
 * the batched adjoint calls below do not (their grids and workspace follow
 * the channel set): replayed after a replan they write nothing, and must
 * be captured again.
 */
sos_status sos_batch_replan(sos_batch_t batch, const sos_plan_t *plans, int32_t C, const int64_t *n,
                            const int64_t *offsets, sos_stream_t stream);

/*
 * sos_batch_query -- the schedule, for inspection and tests.  Every output
 * pointer is host memory and may be NULL.
 * total     samples spanned by the concatenated buffers (max offset + n).
 * items     wavefront work items (4 tiles each) of the launch.
 * offsets   [C]: first sample of each channel.
 * tile      [C]: samples per tile of each channel (a multiple of 16 N).
 * order     [C]: channel indices in launch order (costliest items first).
 */
sos_status sos_batch_query(sos_batch_t batch, int64_t *total, int64_t *items, int64_t *offsets,
                           int64_t *tile, int32_t *order);

/*
 * sos_filt_batched -- y_c = cascade_c(x_c) for every channel, zero initial
 * state, one kernel launch on `stream`.
 *
 * x, y       device, `total` samples of the plans' io_dtype each, channel c
 *            at its offset; 16-byte aligned; must not overlap.  Samples of
 *            y between channels are not written.
 * workspace  unused (NULL).
 * Asynchronous, no allocation, no synchronisation, so it can be captured
 * in a HIP graph.  Calls with one batch may run concurrently.
 */
sos_status sos_filt_batched(sos_batch_t batch, const void *x, void *y, void *workspace,
                            sos_stream_t stream);

/*
 * Reverse-mode gradient (adjoint) of y = cascade(x) for a loss L with
 * upstream gradient gy = dL/dy.  With u_k the input and w_k the output of
 * section k, and A_k, B_k the banded Toeplitz matrices of its denominator
 * and numerator (the matrix form of the recurrence in Section II):
 *   mu_k = A_k^{-T} lambda_k,  lambda_{k-1} = B_k^T mu_k,  lambda_K = gy,
 *   gx = dL/dx = lambda_0,
 *   dL/db_j = sum_i mu_k[i] u_k[i-j],  dL/da_j = -sum_i mu_k[i] w_k[i-j],
 * then the chain rule through the division of each row by its a0.  The
 * transposed filters run backwards in time, so the kernels take the groups
 * in reversed time and reuse the PH solve of Section VI-B for A^{-T}.
 *
 * Two modes, fixed by the plan (SOS_FLAG_ADJ_SAVE, SOS_FLAG_ADJ_RECOMPUTE, or
 * by cost when neither is set):
 *  - saved outputs: the forward pass stores every section's output (FP64,
 *    K n samples) and the adjoint reads them back;
 *  - recompute: the forward pass stores the cascade state (2K + 2 values)
 *    at every group of 256 samples and, for K >= 8, section K/2's input
 *    (FP64, n samples); the adjoint recomputes section k's input in each
 *    group from the nearest kept one below it: the group's input, section
 *    K/2's, and in each half two more kept on that half's first pass, one
 *    in LDS (FP32 I/O, 4 <= K <= 17) and one in registers.  At K = 8 that
 *    is 7 forward section passes per group, where recomputing every input
 *    from the group's state would take K(K-1)/2 + 1 = 29.
 * Measured costs per sample on MI355X, in ps, P the passes per group:
 * saved outputs 4.23 + 3.38 K (FP32 I/O), 7.92 + 3.36 K (FP64 I/O);
 * recompute 2.34 + 1.75 K + 0.331 P (FP32 I/O), 5.38 + 1.57 K + 0.381 P
 * (FP64 I/O), times 1.34 or 1.28 where the adjoint's LDS leaves one
 * wavefront per SIMD.  So without a flag a plan recomputes for K <= 40
 * with FP32 I/O and K <= 31 with FP64 I/O.
 *
 * sos_backward_workspace_size -- device bytes sos_filt_backward needs for n
 * samples: the saved outputs (K n doubles, padded) or the group states
 * ((2K + 2) doubles per 256 samples, and for K >= 8 one double per sample
 * for the kept section input), and the per-tile partial sums.  0 for a
 * host-only plan.
 */
size_t sos_backward_workspace_size(sos_plan_t plan, int64_t n);

/*
 * sos_filt_backward -- gx = dL/dx and gsos = dL/d(sos) for y = cascade(x).
 *
 * x, gy      device, n samples of the plan's io_dtype: the forward input
 *            and dL/dy.
 * gx         device, n samples (io_dtype), written; must not overlap x or gy.
 * gsos       device, [K][6] float64 row-major, written: the gradient with
 *            respect to the caller's rows (b0, b1, b2, a0, a1, a2).
 * n          >= 0; n == 0 writes gsos = 0 only.
 * workspace  device, sos_backward_workspace_size(plan, n) bytes, 16-byte
 *            aligned; its contents on entry do not matter.
 * The adjoint always runs PH with FP64 arithmetic at N = 16, whatever the
 * plan's solver, N and compute dtype (the same cascade, exact to rounding).
 * It first re-runs the forward pass (saving section outputs or group
 * states, as above), so the caller's forward result is not needed.  Sums
 * over the signal are formed per tile and added in a fixed order: results
 * are deterministic.
 */
sos_status sos_filt_backward(sos_plan_t plan, const void *x, const void *gy, void *gx,
                             double *gsos, int64_t n, void *workspace, sos_stream_t stream);

/*
 * A training step in two calls, without the backward's own forward pass.
 * The two calls give the same gx and gsos as sos_filt_backward.
 *
 * sos_filt_for_backward -- the forward pass of sos_filt_backward, which
 * also stores y = cascade(x).  It fills the workspace with what the adjoint
 * needs (section outputs or group states).
 *   x          device, n samples (io_dtype), read.
 *   y          device, n samples (io_dtype), written; must not overlap x.
 *              Computed by the adjoint's path (PH, FP64 arithmetic,
 *              N = 16): sos_filt's result to rounding.
 *   workspace  device, sos_backward_workspace_size(plan, n) bytes, 16-byte
 *              aligned.
 * sos_filt_backward_stored -- the adjoint of sos_filt_backward from that
 * workspace: the same plan, x, n and workspace, left unchanged in between.
 * Other arguments as sos_filt_backward.
 */
sos_status sos_filt_for_backward(sos_plan_t plan, const void *x, void *y, int64_t n, void *workspace,
                                 sos_stream_t stream);
sos_status sos_filt_backward_stored(sos_plan_t plan, const void *x, const void *gy, void *gx,
                                    double *gsos, int64_t n, void *workspace, sos_stream_t stream);

/*
 * Batched adjoint: sos_filt_backward for every channel of a device batch in
 * three launches (the forward pass that saves the section outputs or the
 * group states, the reversed-time adjoint, the reduction of the coefficient
 * sums).  One mode for the whole batch: saved outputs if any channel's plan
 * has SOS_FLAG_ADJ_SAVE, else recompute if any has SOS_FLAG_ADJ_RECOMPUTE,
 * else the cheaper by the costs above summed over the channels' samples.
 *
 * sos_batch_backward_workspace_size -- device bytes of the workspace (0 if
 * the batch has no adjoint: host-only batches).
 * sos_batch_query_adjoint -- rows of gsos (the sum of the channels' K) and,
 * into first_row (host [C] or NULL), each channel's first row.
 * sos_filt_backward_batched -- x, gy: device, the batch's concatenated
 * layout; gx: device, same layout, written at the channels' samples only,
 * must not overlap x or gy; gsos: device float64 [rows][6], channel c's K
 * rows from its first row, with respect to its rows (b0 b1 b2 a0 a1 a2);
 * workspace: device, the size above, 16-byte aligned.  The semantics,
 * precision and determinism are those of sos_filt_backward.
 */
size_t sos_batch_backward_workspace_size(sos_batch_t batch);
sos_status sos_batch_query_adjoint(sos_batch_t batch, int64_t *gsos_rows, int64_t *first_row);
sos_status sos_filt_backward_batched(sos_batch_t batch, const void *x, const void *gy, void *gx,
                                     double *gsos, void *workspace, sos_stream_t stream);
/*
 * The batched training step in two calls, as sos_filt_for_backward and
 * sos_filt_backward_stored.  y has the batch's layout and is written at
 * the channels' samples only.
 */
sos_status sos_filt_batched_for_backward(sos_batch_t batch, const void *x, void *y, void *workspace,
                                         sos_stream_t stream);
sos_status sos_filt_backward_batched_stored(sos_batch_t batch, const void *x, const void *gy, void *gx,
                                            double *gsos, void *workspace, sos_stream_t stream);

/*
 * sos_batch_tune -- autotuner for batches: times sos_filt_batched for every
 * candidate (N, L, tile_groups) on the caller's own buffers and reports the
 * fastest.
 *
 * sos, K     host [C]: channel c's [K[c]][6] coefficient rows (as sos_plan).
 * n, offsets as sos_batch_plan.
 * base       host, may be NULL: dtypes and solver of the plans (its N, L and
 *            tile_groups are ignored).
 * Ns, nN     host: candidate N values; Ls, nL: candidate L values (16, 32,
 *            64); tiles, nt: candidate tile_groups (0 = the library's
 *            choice).
 * x, y       device buffers laid out as the batch (y is overwritten).
 * reps       timed launches per candidate, after untimed launches for at
 *            least 30 ms (code load, clocks after the host-side planning).
 * results    host [nN * nL * nt] or NULL: every candidate's seconds per
 *            launch, N-major, then L.
 * best       host: the fastest candidate.
 * Synchronous: it creates and destroys plans and batches (allocates) and
 * waits for its own launches on `stream`.  Errors from any candidate's plan
 * or launch end the search and are returned.
 */
typedef struct {
    int32_t N;
    int32_t L;
    int32_t tile_groups;
    int32_t reserved;   /* 0 */
    double seconds;
} sos_tune_result;

sos_status sos_batch_tune(const double *const *sos, const int32_t *K, int32_t C, const int64_t *n,
                          const int64_t *offsets, const sos_opts *base, const int32_t *Ns, int32_t nN,
                          const int32_t *Ls, int32_t nL, const int32_t *tiles, int32_t nt, const void *x, void *y,
                          int32_t reps, sos_stream_t stream, sos_tune_result *results, sos_tune_result *best);

const char *sos_status_string(sos_status s);

#ifdef __cplusplus
}
#endif

#endif /* SOSFILT_H */
