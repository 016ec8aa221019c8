/* pc.h -- C ABI of the MI355X product-convolution library.
 *
 * The library applies the adaptive product-convolution approximation of
 * Alger, Rao, Myers, Bui-Thanh and Ghattas (arXiv 1805.06018),
 *
 *     A~ u = sum_k phi_k^E * (w_k . u)                    (eq. (2.5))
 *
 * and its adjoint (eq. (1.6)) to batches of vectors on one AMD Instinct
 * MI355X (gfx950), and drives the randomized a-posteriori error estimator
 * (Sec. 2.6) on top of the adjoint.
 *
 * Conventions
 *  - The domain Omega is the box prod_i [0, shape[i]-1] in Z^d, d in
 *    {1, 2, 3}.  Grid functions are stored row-major over Omega (axis 0
 *    slowest), N = prod shape.
 *  - Boxes are inclusive integer boxes [lo, hi]; arrays of boxes and points
 *    are row-major [count][d] int64.
 *  - Batched vectors are contiguous: vector j of a batch starts at
 *    base + j * ld elements (ld >= N).
 *  - Every pointer named u/U/V/OUT/Z/Y is DEVICE memory owned by the caller;
 *    every other pointer is HOST memory owned by the caller and only read
 *    during the call (pc_create deep-copies what it needs).
 *  - Calls are asynchronous on the given HIP stream unless stated; nothing
 *    throws across the ABI; a failing call returns a status and sets a
 *    thread-local message readable with pc_last_error().
 *  - An operator is read-only after pc_create.  Calls on one operator must be
 *    serialised by the caller (they share the operator's work buffers:
 *    staging, 3-D scratch, estimator buffers, the unit counters of the
 *    persistent launch); different operators are
 *    independent.  A call whose work buffers must grow releases the old ones
 *    in stream order after the operator's previous call has ended (an event;
 *    neither the host nor other streams wait) and allocates on its stream.
 *  - Graph capture: pc_apply, pc_apply_batch, pc_apply_adjoint_batch,
 *    pc_apply_batch_plain, the two _axpy calls and pc_entries only launch
 *    kernels on s once the operator's work buffers are large enough, so a
 *    caller may record them into a HIP graph by stream capture after one
 *    call of at least the same batch size (same entry point and tuning)
 *    outside the capture.  A captured call whose buffers would have to grow
 *    returns PC_ERR_ARG without enqueuing anything.  The graph replays with
 *    the pointers given at capture and keeps using the operator's buffers:
 *    replays must not overlap other calls on the same operator, and a later
 *    call that needs larger buffers frees the old ones, after which graphs
 *    recorded earlier must not be replayed.
 *    pc_apply_block, pc_estimate_sums and pc_error_estimate synchronise the
 *    host and return PC_ERR_ARG under capture.
 */
#ifndef PC_H_
#define PC_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pc_op pc_op;

typedef enum {
    PC_OK = 0,
    PC_ERR_ARG = 1,          /* invalid argument (null pointer, bad size, bad radius) */
    PC_ERR_GRID = 2,         /* leaves do not tile Omega, or points != sorted corners  */
    PC_ERR_OOM = 3,          /* device or host allocation failed                       */
    PC_ERR_BUDGET = 4,       /* request exceeds a configured memory budget             */
    PC_ERR_DEVICE = 5,       /* a HIP call failed; destroy the operator                */
    PC_ERR_CALLBACK = 6,     /* the user's exact-adjoint callback returned non-zero    */
    PC_ERR_UNSUPPORTED = 7   /* valid input outside what the library implements       */
} pc_status;

typedef enum { PC_F32 = 0, PC_F64 = 1 } pc_dtype;

/* Extend impulse responses by zero instead of by the neighbour average of
 * Sec. 2.5 (the plain scheme whose boundary artifacts Fig. 2 shows). */
#define PC_NO_EXTEND (1u << 0)

/* Plan 1-D/2-D work items within half of a CU's LDS (80 KB) and run them in
 * 512-thread workgroups, two per CU, instead of up to 160 KB in 1024-thread
 * workgroups (FP32; FP64 items always use 512 threads).  Same results to
 * rounding; a scheduling choice. */
#define PC_PLAN_HALF_LDS (1u << 1)

/* 1-D/2-D plans: the smallest supported FFT lengths, pieces by the least
 * n log n.  By default the planner picks lengths up to 35 % longer where a
 * cheaper radix factorisation and the staged output volume give a lower
 * estimated time (instruction counts of the compiled codelets).  Same
 * results to rounding; a scheduling choice. */
#define PC_PLAN_SMALLEST_FFT (1u << 2)

/* pc_create -- build the operator (Sec. 2.2, 2.4, 2.5) and its device data.
 *
 *  d, shape[d]          : Omega.
 *  n_leaves, leaf_lo/hi : the leaf cells of the adaptive cell tree (Sec. 2.2),
 *                         [n_leaves][d] inclusive boxes.  They must tile Omega
 *                         (interiors disjoint, union = Omega), else PC_ERR_GRID.
 *  r, points[r][d]      : the sample points p_k = sorted (axis 0 most
 *                         significant) union of all leaf corners, else
 *                         PC_ERR_GRID.  Index k of a point is its position.
 *  radius[r][d]         : phi_k is supplied on the box prod_i [-R_ki, R_ki]
 *                         (R >= 0, else PC_ERR_ARG).
 *  phi, phi_off[r+1]    : the impulse responses phi_k[z] = (A delta_{p_k})[z+p_k]
 *                         (eq. (2.6)), concatenated: patch k occupies
 *                         phi[phi_off[k] .. phi_off[k+1]) = prod (2R_ki+1)
 *                         doubles, row-major with offset z = -R first.
 *                         Entries with p_k + z outside Omega are ignored;
 *                         phi_k is taken as 0 outside the supplied box.
 *  dtype                : arithmetic of the apply (FP32 or FP64).  Setup is
 *                         FP64; the spectra are rounded once to dtype.
 *  flags                : PC_NO_EXTEND, PC_PLAN_HALF_LDS, PC_PLAN_SMALLEST_FFT, or 0.
 *  s                    : stream of the uploads (synchronised before return;
 *                         no device-wide synchronisation).
 *  out                  : receives the operator.
 * Weights w_k are the harmonic partition of unity of Sec. 2.4: multilinear
 * hats on cells without hanging nodes; on cells with hanging nodes the
 * discrete harmonic extension, recursively in dimension (edges cut at the
 * points on them, facets - a broken 3-D facet as the facets of the smaller
 * leaves on its other side - then the cell), solved exactly.
 * PC_ERR_UNSUPPORTED is returned when a patch's FFT box exceeds the
 * kernels' limits (FFT lengths up to 256 along axis 0 (and axis 1 in 3-D),
 * real length up to 256 along the last axis, one LDS-resident plane per
 * workgroup; 2-D patches are cut into pieces, 3-D ones are not).
 */
pc_status pc_create(int d, const int64_t* shape,
                    int64_t n_leaves, const int64_t* leaf_lo, const int64_t* leaf_hi,
                    int64_t r, const int64_t* points, const int64_t* radius,
                    const double* phi, const int64_t* phi_off,
                    pc_dtype dtype, uint32_t flags, hipStream_t s, pc_op** out);

/* pc_create_patches -- the operator restricted to a subset S of the terms of
 * the sum (eq. (2.5)):  A~_S u = sum_{k in S} phi_k^E * (w_k . u),  with w_k
 * and phi_k^E those of the full tiling (arguments as pc_create).  It serves
 * the incremental update of Y~ = A~* Z during refinement (Sec. 2.8): only the
 * terms of new points and of points whose cells, weights or neighbours
 * changed are convolved again.  sel[n_sel]: distinct point indices in [0, r)
 * (host, any order); n_sel = 0 gives the zero operator; n_sel < 0 or an
 * index out of range or repeated gives PC_ERR_ARG.  Only the selected
 * patches' weights, spectra and work items are built and held. */
pc_status pc_create_patches(int d, const int64_t* shape,
                            int64_t n_leaves, const int64_t* leaf_lo, const int64_t* leaf_hi,
                            int64_t r, const int64_t* points, const int64_t* radius,
                            const double* phi, const int64_t* phi_off,
                            pc_dtype dtype, uint32_t flags, int64_t n_sel, const int64_t* sel,
                            hipStream_t s, pc_op** out);

/* pc_apply -- out = A~ u for one vector (eq. (2.5)).  u, out: device, N
 * elements of the operator's dtype; out must not alias u. */
pc_status pc_apply(pc_op* op, const void* u, void* out, hipStream_t s);

/* pc_apply_batch -- OUT[:, j] = A~ U[:, j] for j < B (eq. (2.5)), all vectors
 * in one fused launch sequence.  U and OUT are device arrays with leading
 * dimensions ldu, ldo >= N; B >= 0 (B = 0 is a no-op). */
pc_status pc_apply_batch(pc_op* op, int64_t B, const void* U, int64_t ldu,
                         void* OUT, int64_t ldo, hipStream_t s);

/* pc_apply_adjoint_batch -- OUT[:, j] = A~* V[:, j] (eq. (1.6): the same
 * patches in reverse order, convolution with the flipped kernel first, then
 * the weight). */
pc_status pc_apply_adjoint_batch(pc_op* op, int64_t B, const void* V, int64_t ldv,
                                 void* OUT, int64_t ldo, hipStream_t s);

/* pc_apply_batch_plain -- same result as pc_apply_batch, computed the plain
 * way: one launch per patch and per vector, outputs summed in the same
 * order.  Kept as the baseline the fused path is measured against. */
pc_status pc_apply_batch_plain(pc_op* op, int64_t B, const void* U, int64_t ldu,
                               void* OUT, int64_t ldo, hipStream_t s);

/* pc_apply_batch_noalloc -- pc_apply_batch for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and the same result,
 * bit for bit, as pc_apply_batch.  Instead of the operator's grown work
 * buffers it uses a fixed work area of 128 MiB per device, set up by the
 * first pc_create on that device and held until the process ends; it
 * allocates and frees nothing and creates no HIP objects.  Vectors run in
 * chunks whose staging fits the area (3-D operators: one vector at a time,
 * its staging plus the plane scratch of each item group).  An operator
 * whose staging for one vector (or, in 3-D, one item's scratch beside it)
 * does not fit returns PC_ERR_UNSUPPORTED before anything is enqueued; the
 * 1024^2 blur with ~600 points needs 65 MB per vector in FP32.  All calls
 * on one device share the area and each call leaves its contents behind:
 * calls that may overlap on the device (different streams, or a replayed
 * graph beside an eager call) race and must be serialised by the caller. */
pc_status pc_apply_batch_noalloc(pc_op* op, int64_t B, const void* U, int64_t ldu,
                                 void* OUT, int64_t ldo, hipStream_t s);

/* pc_apply_batch_axpy / pc_apply_adjoint_batch_axpy -- OUT[:, j] += alpha *
 * A~ U[:, j] (eq. (2.5)) or OUT[:, j] += alpha * A~* V[:, j] (eq. (1.6)):
 * the deterministic patch sum of every output point is formed first, then
 * scaled by alpha (rounded to the operator's dtype) and added to OUT once.
 * OUT must not alias the input.  Used to update Y~ in place with the terms
 * of a pc_create_patches operator (alpha = -1 for the old terms, +1 for the
 * new ones). */
pc_status pc_apply_batch_axpy(pc_op* op, int64_t B, const void* U, int64_t ldu, double alpha,
                              void* OUT, int64_t ldo, hipStream_t s);
pc_status pc_apply_adjoint_batch_axpy(pc_op* op, int64_t B, const void* V, int64_t ldv, double alpha,
                                      void* OUT, int64_t ldo, hipStream_t s);

/* Exact adjoint matvec supplied by the caller: out[:, j] = A* in[:, j] for
 * j < B on stream s (device arrays of the operator's dtype).  Return 0 on
 * success; any other value aborts the estimate with PC_ERR_CALLBACK. */
typedef int (*pc_matvec_fn)(void* user, int64_t B, const void* in, int64_t ldin,
                            void* out, int64_t ldout, hipStream_t s);

/* pc_error_estimate -- randomized estimator of Sec. 2.6 (eq. (2.11)).
 *  Z [q][ldz]         : probe vectors (device).
 *  Y_or_null [q][ldy] : Y = A* Z if the caller has it (computed once and
 *                       reused, Sec. 2.8); if NULL the library calls
 *                       exact_adjoint to fill a work buffer.
 *  eta_leaf[n_leaves] : host output or NULL; eta_C = q^{-1/2} ||(Y~ - Y)[C, :]||_F
 *                       with C's own points (shared facets count in each cell).
 *  eta_abs            : host output, q^{-1/2} ||Y~ - Y||_F.
 *  eta_rel            : host output, ||Y~ - Y||_F / ||Y||_F.
 * Y~ and Y are promoted to FP64 before they are subtracted, and all sums of
 * squares are accumulated in FP64 in a fixed order.  Synchronises s before
 * returning.  The operator stays valid after PC_ERR_CALLBACK. */
pc_status pc_error_estimate(pc_op* op, int64_t q, const void* Z, int64_t ldz,
                            const void* Y_or_null, int64_t ldy,
                            pc_matvec_fn exact_adjoint, void* user,
                            double* eta_leaf, double* eta_abs, double* eta_rel,
                            hipStream_t s);

/* pc_apply_block -- apply a block of the operator (Sec. 3.3):
 *   adjoint = 0:  OUT_T[:, j] = A~[T, S] U_S[:, j]
 *   adjoint = 1:  OUT_T[:, j] = A~*[T, S] U_S[:, j]  ((A~*)[T, S] = A~[S, T]*)
 * tlo/thi, slo/shi: host int64 [d] inclusive boxes inside Omega (else
 * PC_ERR_ARG).  U_S: device [B][ldu], each vector row-major over the box S
 * (ldu >= |S|); OUT_T: device [B][ldo] over T (ldo >= |T|), fully written.
 * Only the work items whose gather box meets S (adjoint: whose output box
 * meets S) and whose written box meets T run, both boxes clipped, so the
 * cost follows the paper's O(r_S sigma log sigma) (adjoint: r_T).  Results
 * equal the restriction to T of the full apply to U_S extended by zero.
 * Each call copies its small tables to the device synchronously. */
pc_status pc_apply_block(pc_op* op, int adjoint, const int64_t* tlo, const int64_t* thi,
                         const int64_t* slo, const int64_t* shi, int64_t B,
                         const void* U, int64_t ldu, void* OUT, int64_t ldo, hipStream_t s);

/* pc_entries -- matrix entries out[i] = A~[ys[i], xs[i]] for i < n (Sec. 3.1,
 * eq. (3.1)): sum over the points k of a leaf containing x of
 * w_k[x] phi_k^E[y - x], accumulated in FP64 in ascending k and rounded to
 * the operator's dtype (weights and kernels are held in that dtype).
 * ys, xs: device int64 [n][d] Omega coordinates; out: device [n] of the
 * operator's dtype.  A pair with y or x outside Omega gives NaN.  For an
 * operator from pc_create_patches only the kept terms are summed.  The
 * first call uploads the entry tables (a leaf index per grid point and the
 * extended kernels, about N * 4 bytes plus the kernels in dtype), kept until
 * pc_destroy. */
pc_status pc_entries(pc_op* op, int64_t n, const int64_t* ys, const int64_t* xs,
                     void* out, hipStream_t s);

/* pc_estimate_sums -- the estimator of Sec. 2.6 (eq. (2.11)) from a Y~ the
 * caller already holds (e.g. updated incrementally with the axpy calls):
 * eta_leaf[c] = sqrt(sum_{x in C} sum_i (Y~ - Y)^2 / q) over the operator's
 * leaves, eta_abs, eta_rel as pc_error_estimate.  Yt, Y: device [q][ldt],
 * [q][ldy] of the operator's dtype; host outputs written after the stream
 * is synchronised. */
pc_status pc_estimate_sums(pc_op* op, int64_t q, const void* Yt, int64_t ldt,
                           const void* Y, int64_t ldy, double* eta_leaf,
                           double* eta_abs, double* eta_rel, hipStream_t s);

/* pc_estimate_sums_device -- the sums behind the estimator of Sec. 2.6
 * (eq. (2.11)), left on the device in stream order, for callers that must
 * not block (a serving loop reads them after an event):
 *   sums[c]            = sum_{x in C} sum_i (Y~ - Y)^2 for each leaf c,
 *   sums[n_leaves]     = sum over Omega (each point once) of (Y~ - Y)^2,
 *   sums[n_leaves + 1] = sum over Omega of Y^2,
 * FP64, in the fixed order of pc_estimate_sums, whose outputs follow as
 * eta_C = sqrt(sums[c] / q), eta_abs = sqrt(sums[L] / q), eta_rel =
 * sqrt(sums[L] / sums[L + 1]).  sums: device double[n_leaves + 2], caller
 * owned.  Does not synchronise; capturable once the operator's estimator
 * buffer exists (after one estimator call outside the capture). */
pc_status pc_estimate_sums_device(pc_op* op, int64_t q, const void* Yt, int64_t ldt,
                                  const void* Y, int64_t ldy, double* sums, hipStream_t s);

/* Plan statistics (for measurement and admission). */
typedef struct {
    int64_t n;              /* N = |Omega|                                          */
    int64_t r;              /* number of sample points                              */
    int64_t n_leaves;
    int64_t n_items;        /* convolution work items (patches, or patch pieces)    */
    int64_t sum_fft_points; /* sum over items of the FFT box size                   */
    double  alg_flops_per_rhs;  /* 5 n log2 n + 3 n + |I| + |O| summed, n = FFT box */
    int64_t kernel_elems;   /* sum over patches of the extended kernel box size     */
    int64_t spectrum_bytes; /* resident spectra                                     */
    int64_t weight_bytes;   /* resident weight tables                               */
    int64_t slot_elems_fwd; /* per-vector staging elements of the forward apply     */
    int64_t slot_elems_adj; /* per-vector staging elements of the adjoint apply     */
    int64_t device_bytes;   /* everything resident except per-call work buffers     */
    int32_t dtype;
    int32_t max_lds_bytes;  /* largest LDS footprint of an item                     */
} pc_stats;

pc_status   pc_get_stats(const pc_op* op, pc_stats* st);

/* Kernel timing for measurement.  pc_set_profiling(op, 1) makes every later
 * apply (not under stream capture) time each convolution and each reduction
 * launch with a HIP event pair: in staged 1-D/2-D applies the events travel
 * on the launch's own dispatches (start with its first kernel, stop with its
 * last), elsewhere they are recorded on the stream around the launch.
 * pc_read_profile waits for those events, returns the accumulated device
 * times and launch counts since the last read, and resets them.  Timing
 * costs the stream a few microseconds per launch.  Profiling is off after
 * pc_create. */
typedef struct {
    double  conv_ms;          /* summed duration of the convolution launches  */
    double  reduce_ms;        /* summed duration of the reduction launches    */
    int64_t conv_launches;
    int64_t reduce_launches;
    int64_t conv_vectors;     /* vectors processed by those convolution launches */
} pc_profile;

pc_status   pc_set_profiling(pc_op* op, int enable);

/* pc_debug_fail_launches -- failure injection for tests of a caller's error
 * handling (no GPU fault is involved).  Counting the operator's convolution
 * launches from 1 after this call, launches first .. first + count - 1 fail
 * with PC_ERR_DEVICE before anything of theirs is enqueued; earlier
 * launches of the same call may have run, so its outputs are undefined.
 * Unlike a real device error, an injected one leaves the operator usable.
 * count = 0 disables (first is then ignored); otherwise first >= 1, else
 * PC_ERR_ARG.  The environment variable PC_DEBUG_FAIL_LAUNCH=n, read by
 * pc_create and pc_create_patches, has the effect of (n, 1). */
pc_status   pc_debug_fail_launches(pc_op* op, int64_t first, int64_t count);

/* Schedule knobs (defaults chosen by the library; an autotuner may override).
 *  PC_TUNE_CHUNK    vectors per convolution launch (0 = library default:
 *                   as many as fit a 2 GiB staging buffer, 8 GiB for 3-D
 *                   operators; 3-D operators take an explicit value even
 *                   beyond that size)
 *  PC_TUNE_OVERLAP  1: reduce chunk i on a library stream while chunk i+1
 *                   convolves; 0: everything on the caller's stream
 *                   (2-D operators only)
 *  PC_TUNE_SCRATCH  3-D operators: bytes of plane-spectrum scratch per item
 *                   group (0 = library default: 1 GiB in FP32, 256 MiB in
 *                   FP64); one item group runs its three kernels before the
 *                   next group starts
 *  PC_TUNE_DIRECT   1-D/2-D operators, pc_apply_batch and the adjoint: 1
 *                   runs the items colour by colour - the items of one
 *                   colour write pairwise disjoint boxes - and adds each box
 *                   straight into the outputs, which are zeroed first;
 *                   0 (default) stages every item's box and sums them in a
 *                   reduction launch.  Both sum each output point's contributions in
 *                   the same order (ascending colour, then item), so the
 *                   bits are the same.  The axpy forms, block applies and the
 *                   plain path always stage.
 *  PC_TUNE_STREAMS  colour launches: the batch is cut into vector chunks
 *                   (PC_TUNE_CHUNK vectors, default B / streams) whose
 *                   colour sequences run on up to this many library streams
 *                   at once, forked from and joined back into the caller's
 *                   stream with events (1..4, default 4); each chunk keeps
 *                   its own colour order, so the bits do not change
 *  PC_TUNE_BUDGET   cap, in bytes, on the work buffers the operator may hold
 *                   (staging, scratch, estimator and block buffers; 0 = no
 *                   cap): a call that would grow them beyond it returns
 *                   PC_ERR_BUDGET before anything is enqueued
 *  PC_TUNE_PERSISTENT  staged 1-D/2-D applies (pc_apply_batch and the
 *                   adjoint): 1 runs each vector chunk's convolution as a
 *                   fixed grid of workgroups that take (item, vector) units
 *                   from per-XCD queues in device memory (cleared by a
 *                   kernel before each launch) instead of one workgroup per
 *                   unit; 0 (default) launches one workgroup per unit.
 *                   Ignored where the item data leaves no room in LDS for
 *                   the queue slot, and by the other entry points.
 *  PC_TUNE_XCD_ORDER  staged 1-D/2-D applies, one workgroup per unit: 0
 *                   (default) gives each of the 8 XCDs whole items with all
 *                   their vectors (a patch's spectrum stays in one XCD's
 *                   L2); 1 deals the workgroups item-major, so the vectors
 *                   of one item run on all XCDs at once.
 *  PC_TUNE_SPLIT    staged FP32 applies, one workgroup per unit, whole items
 *                   per XCD: 1 (default) runs the items whose FFT box and
 *                   twiddles take at most 79 KiB of LDS as a second launch
 *                   of 512-thread workgroups, two per CU, after the others;
 *                   0 runs all items as 1024-thread workgroups, one per CU.
 * Results are bitwise identical for every setting. */
enum { PC_TUNE_CHUNK = 1, PC_TUNE_OVERLAP = 2, PC_TUNE_SCRATCH = 3, PC_TUNE_BUDGET = 4, PC_TUNE_DIRECT = 5,
       PC_TUNE_STREAMS = 6, PC_TUNE_PERSISTENT = 7, PC_TUNE_XCD_ORDER = 8, PC_TUNE_SPLIT = 9 };
pc_status   pc_set_tuning(pc_op* op, int key, int64_t value);
pc_status   pc_read_profile(pc_op* op, pc_profile* out);
/* pc_device_bytes -- device bytes the operator holds now: its resident data
 * (spectra, weights, tables) plus the work buffers grown by earlier calls
 * (staging, 3-D scratch, estimator buffers), which it keeps until
 * pc_destroy.  For HBM-budget admission; 0 for a null operator. */
size_t      pc_device_bytes(const pc_op* op);
pc_status   pc_destroy(pc_op* op);
const char* pc_status_string(pc_status st);
const char* pc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PC_H_ */
