/*
 * rsd.h -- C interface of the recursive-skeletonisation direct solver for
 * 2-D volume integral equations on MI355X (gfx950).
 *
 * Method: Corona, Martinsson, Zorin, "An O(N) Direct Solver for Integral
 * Equations on the Plane".  The solver builds a compressed inverse of the
 * Nystrom matrix of
 *     a(x) s(x) + int_Omega b(x) K(|x - y|) c(y) s(y) dy = f(x)
 * (Sec. 5, general formulation) on a regular grid, level by level over the
 * binary tree of Sec. 2.2, with boundary-layer skeletons (Sec. 3.1), proxy
 * interpolation (Sec. 2.2, Sec. 3.3.2) and the inverse of Algorithm 1 in the
 * block form of Algorithm 2, and applies it with Algorithm 6.
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major.  A block of right-hand sides is N x nrhs with
 *     leading dimension N (column c starts at element c * N).
 *   - Pointers may be host or device memory (detected per call).  Inputs are
 *     borrowed for the duration of the call only; the factor owns copies of
 *     everything it keeps.  Outputs are written by the library into memory
 *     the caller allocated.
 *   - Every function returns an rsd_status; on failure a description is
 *     available from rsd_last_error() (thread-local) and output handles are
 *     set to NULL.  No C++ exception crosses this interface.
 *   - Complex data (Helmholtz kernel) is interleaved (re, im) double pairs.
 */
#ifndef RSD_H
#define RSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rsd_status {
    RSD_OK = 0,
    RSD_EINVAL = 1,     /* bad argument: NaN/Inf input, tol <= 0, nrhs < 0, ... */
    RSD_ENOTGRID = 2,   /* points are not a complete uniform grid (Sec. 2.2) */
    RSD_ENOMEM = 3,     /* device memory exhausted or over the caller's budget */
    RSD_ESINGULAR = 4,  /* a pivot block was singular; message names level/box */
    RSD_ENOCONV = 5,    /* iterative refinement did not reach its tolerance */
    RSD_EDEVICE = 6,    /* HIP runtime error */
    RSD_EAGAIN = 7      /* not finished within the timeout / no capacity now */
} rsd_status;

typedef enum rsd_kernel_type {
    RSD_KERNEL_LAPLACE = 0,   /* K(r) = (1/2pi) log r                         */
    RSD_KERNEL_HELMHOLTZ = 1  /* G(r) = (i/4) H0^(1)(k r), outgoing solution   */
} rsd_kernel_type;

/* Kernel of the integral operator.  With contrast_b == NULL the matrix is
 *   A_ij = a_i delta_ij + h^2 K(|x_i - x_j|)        (i != j),
 *   A_ii = a_i + int_{cell_i} K(|x_i - y|) dy,
 * the Nystrom rule of Sec. 5 with b = c = 1 and the exact integral of the
 * kernel over the point's own cell on the diagonal.  With contrast_b given
 * (N values, b > 0 at every point; a must be NULL) it is the scattering
 * operator of Sec. 5.4:
 *   A_ij = sqrt(b_i) h^2 G(|x_i - x_j|) sqrt(b_j),  A_ii = 1 + b_i int_cell G,
 * factored as S M S with S = diag(sqrt b) and M = diag(1/b) + h^2 G (whose
 * off-diagonal part is translation invariant); zero or negative b => EINVAL.
 * The Helmholtz kernel (wavenumber > 0) makes the matrix complex symmetric:
 * the factor holds the real symmetric form [[Re, Im], [Im, -Re]] of every
 * block on two dofs per point, and right-hand sides and solutions are
 * interleaved complex doubles.  Batched builds take the Laplace kernel
 * without a contrast only (EINVAL otherwise). */
typedef struct rsd_kernel {
    int32_t type;              /* rsd_kernel_type                           */
    double wavenumber;         /* k of the Helmholtz kernel; ignored else   */
    const double* contrast_b;  /* N values in the caller's point order, or NULL */
} rsd_kernel;

typedef enum rsd_precision {
    RSD_PREC_FP64 = 0,         /* every level in float64                    */
    RSD_PREC_FP32_REFINE = 1   /* levels in float32, root block in float64,
                                  float64 residual + iterative refinement   */
} rsd_precision;

/* Options; an all-zero struct selects the defaults. */
typedef struct rsd_options {
    int32_t leaf_side;     /* largest leaf side in points; 0 => 8               */
    int32_t layers;        /* skeleton/proxy layers m; 0 => from tol:
                              1 if tol >= 1e-6, 2 if tol >= 1e-11, else 3      */
    int32_t precision;     /* rsd_precision                                    */
    int32_t max_refine;    /* refinement steps per solve; 0 => 10 for
                              FP32_REFINE, none for FP64; < 0 => none          */
    double refine_tol;     /* target relative residual; 0 => tol               */
    void* hip_stream;      /* hipStream_t to run on; NULL => a library stream  */
    int32_t device;        /* HIP device ordinal; < 0 => the current device    */
    int32_t flags;         /* RSD_FLAG_* bits                                  */
    double interface_ppw;  /* Helmholtz kernel: skeleton points per wavelength
                              kept on the cut between the children of every
                              box above the leaves (Sec. 5.3: needed as the
                              wavenumber grows), spaced floor(2 pi / (k h
                              ppw)) grid cells apart on the two grid lines
                              beside the cut; 0 => none; ignored for Laplace */
} rsd_options;

/* Keep every box's E_i block after the build (for inspection). */
#define RSD_FLAG_KEEP_E 1
/* Solve every interpolation problem whole, without splitting mirror-symmetric
 * box types into their symmetry sectors (two or four; same T up to rounding
 * for full-rank problems; for testing and comparison). */
#define RSD_FLAG_NO_SYMMETRY 2
/* FP32_REFINE factors: solve the interpolation problems of the float32 levels
 * in float32 too, truncated at max(tol, 1e-6).  By default they are solved in
 * float64 (truncated at min(tol, 1e-10) with two skeleton layers, min(tol,
 * 1e-12) with three, tol with one; symmetry split where full rank) and T is
 * rounded to float32;
 * the float32 form trades interpolation accuracy for a float32-only build and
 * usually needs more refinement steps. */
#define RSD_FLAG_FP32_INTERP 4
/* Build every box's blocks even when the diagonal coefficient a is constant
 * (by default such a factor keeps one E/G/W block per box type and level,
 * shared by all its boxes: the translation-invariant case of Sec. 5.1.2). */
#define RSD_FLAG_NO_DEDUP 8
/* Capture the up sweep, root and down sweep of each solve width once into a
 * HIP graph and replay it (same kernels, same results; needs a non-blocking
 * stream, else the sweeps are launched one by one).  On MI355X at 256^2 with
 * 16 right-hand sides the replay is no faster than the launches one by one
 * (their own durations bound the sweeps), so it is off by default; it helps
 * callers whose host thread is the bottleneck of launch submission. */
#define RSD_FLAG_SOLVE_GRAPH 16
/* Solve the interpolation problems with truncation only.  By default, where
 * truncation would decide the rank (three skeleton layers in float64, and
 * float32 interpolation), they are solved as damped least squares instead,
 * min |K(Z, X^sk) T - K(Z, X^rs)|^2 + (tol |R_11|)^2 |T|^2 (tol: max(tol,
 * 1e-6) in float32), by the same QR on k more rows: the window pivoting
 * decides truncation per sub-panel and stops earlier than column pivoting
 * over all columns, the damped problem has no pivot below tol |R_11| and
 * bounds T.  For comparison and testing. */
#define RSD_FLAG_NO_DAMPING 32

typedef struct rsd_solve_info {
    int32_t refine_iters;  /* refinement steps taken                          */
    double rel_residual;   /* max over columns of |f - A x| / |f| (exact,
                              float64), or -1 when no residual was computed    */
} rsd_solve_info;

typedef struct rsd_factor rsd_factor;

/* Build the compressed inverse (Algorithm 1 in the form of Algorithm 2,
 * fine-to-coarse over the tree of Sec. 2.2).
 *   points  N x 2 row-major (x, y) coordinates of a complete uniform grid in
 *           any order (the solver permutes internally; results come back in
 *           this order).
 *   a       N identity-term coefficients a(x_i) in point order; NULL => 1.
 *           Ignored when kernel->contrast_b is set (then a = 1).
 *   tol     local truncation tolerance of every compression (Sec. 5.1), > 0.
 *   opt     NULL => defaults.
 *   out     receives the factor; free it with rsd_free.
 * Errors: EINVAL, ENOTGRID, ENOMEM, ESINGULAR, EDEVICE.  The call returns
 * after the factor is complete on the device. */
rsd_status rsd_build_factor(const double* points, int64_t n_points,
                            const rsd_kernel* kernel, const double* a,
                            double tol, const rsd_options* opt,
                            rsd_factor** out);

/* Several independent factorizations in one call (many grids of uneven size,
 * e.g. a batch of small problems).  Instance i is the factor
 * rsd_build_factor(points[i], n_points[i], kernel, a[i], tol, opt, &out[i])
 * would build: the same interpolation matrices bit for bit, and the same
 * level arithmetic up to the order of rounding (merged products may split
 * their K ranges differently).  The instances are built in groups of
 * max_inflight (<= 0 => 64): the interpolation problems of every box type of
 * a group are solved together (one launch per window serves all of them),
 * then every level, counted from the leaves, runs as one launch per kernel
 * over the boxes of all instances of the group.
 *   points, n_points, a  arrays of n_inst entries (a may be NULL => all 1;
 *                        a[i] may be NULL).  Host or device pointers.
 *   opt                  shared by all instances; opt->hip_stream must be NULL.
 *   out                  n_inst entries; on success each holds a factor to be
 *                        freed with rsd_free.  On any error every out[i] is
 *                        NULL, nothing leaks, and rsd_last_error names the
 *                        failing instance.
 * Errors: as rsd_build_factor, plus EINVAL for n_inst <= 0 or a stream in opt.
 * Returns after every factor is complete on the device. */
rsd_status rsd_build_factor_batched(int32_t n_inst, const double* const* points,
                                    const int64_t* n_points, const rsd_kernel* kernel,
                                    const double* const* a, double tol, const rsd_options* opt,
                                    int32_t max_inflight, rsd_factor** out);

/* x = A^{-1} rhs with the compressed inverse (Algorithm 6), followed by
 * float64 iterative refinement when the factor was built with
 * RSD_PREC_FP32_REFINE (or max_refine > 0).
 *   rhs, x  N x nrhs column-major, caller's point order; real double for the
 *           Laplace kernel, interleaved complex double for Helmholtz.
 *   info    NULL or receives refinement statistics.
 * Errors: EINVAL (NaN/Inf in rhs, nrhs < 0), ENOCONV (refinement did not
 * reach refine_tol; x then holds the last iterate and info the residual),
 * EDEVICE.  Concurrent calls on one factor are safe and run one after the
 * other (a factor has one set of solve vectors and one stream); separate
 * factors are solved concurrently from separate threads, each on its own
 * stream. */
rsd_status rsd_solve(rsd_factor* f, const double* rhs, int64_t nrhs,
                     double* x, rsd_solve_info* info);

/* Solves with several factors in one call: for every instance i,
 * rsd_solve(factors[i], rhs[i], nrhs, x[i], info ? &info[i] : NULL), with the
 * same results; the solves run on up to 8 host threads, each factor on its
 * own stream, so that small solves and their refinement round trips overlap.
 *   factors, rhs, x  arrays of n entries; the factors must be distinct.
 *   info             NULL or n entries.
 * Errors: EINVAL (n <= 0, a null or repeated factor: nothing is solved);
 * otherwise every instance is attempted and the status of the first failing
 * one (in instance order) is returned, with rsd_last_error naming it. */
rsd_status rsd_solve_batched(int32_t n, rsd_factor* const* factors,
                             const double* const* rhs, int64_t nrhs,
                             double* const* x, rsd_solve_info* info);

/* y = A x with the exact Nystrom matrix in float64 (Sec. 5 general
 * formulation; no compression), same layouts as rsd_solve; the product the
 * refinement residual uses.  The off-diagonal part is a Toeplitz-block-
 * Toeplitz product, computed by circulant embedding in a 2-D FFT of size
 * Mx x My (powers of two >= 2 nx, 2 ny) when both are at most 4096, else by
 * a direct sum over all pairs.  Both agree with the direct sum to rounding
 * (relative 1e-13).  Device work space: 3 N nrhs doubles plus the FFT
 * fields, allocated per call. */
rsd_status rsd_matvec(rsd_factor* f, const double* x, int64_t nrhs, double* y);
/* ---- tile autotuner (batched builds, row a10) ------------------------------
 * The grouped GEMM launches of the factor levels pick a tile width (64 or 128)
 * and a split-K target per launch shape bucket (element size, log2 of the
 * 64-wide tile count, of the longest K and of the flops).  rsd_autotune
 * builds the given instances (one rsd_build_factor, or one
 * rsd_build_factor_batched call for n_inst > 1) reps times under each of six
 * candidates, times every tuned launch with HIP events, and keeps for each
 * bucket seen under all candidates the fastest one; later builds in this
 * process use the table (buckets not in it use the built-in rule).  Results
 * differ from untuned builds only by rounding (split-K changes the order of
 * partial sums).  *n_entries receives the number of buckets set.  The table
 * is saved and loaded as text (rsd_tune_save / rsd_tune_load; the file named
 * by the environment variable RSD_TUNE_FILE is loaded at the first build).
 * Tuning is not thread safe with concurrent builds in the same process. */
rsd_status rsd_autotune(int32_t n_inst, const double* const* points, const int64_t* n_points,
                        const rsd_kernel* kernel, const double* const* a, double tol, const rsd_options* opt,
                        int32_t reps, int32_t* n_entries);
rsd_status rsd_tune_save(const char* path);
rsd_status rsd_tune_load(const char* path);
/* Empties the table (builds use the built-in rule again). */
rsd_status rsd_tune_clear(int64_t* n_entries_before);

/* y ~ A x through the factor's own skeletonization (Sec. 2.3: the matrix in
 * recursive-skeleton form, A = D + L A~ R telescoped over the tree), in O(N)
 * work: skeleton charges x^ = x_sk + T x_rs up the tree, at every box above
 * the leaves the kernel block between its two children's skeletons applied
 * to the sibling's charges (kernel values generated on the fly), the
 * potentials spread down as [p; T^T p], and the dense leaf blocks.  Accurate
 * to the factor's interpolation (about tol relative; T in float32 on the
 * float32 levels of an FP32_REFINE factor).  Laplace factors without a
 * contrast (EINVAL otherwise); same layouts as rsd_matvec (host or device,
 * caller's point order); work space 2 N nrhs + 3 V nrhs doubles (V: the
 * total active-set length over the boxes, about 2 N), allocated per call;
 * returns after the factor's stream completes. */
rsd_status rsd_matvec_compressed(rsd_factor* f, const double* x, int64_t nrhs, double* y);

/* rsd_matvec without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same product and result as rsd_matvec; x and y
 * must be device buffers (N x nrhs column-major, caller's point order;
 * EINVAL for host pointers).  Its work space (2 N nrhs doubles plus the FFT
 * spectrum and field, 3 Mx My doubles; or N doubles of kernel table on the
 * direct-sum path) lives in one 64 MiB device array per GPU, held from the
 * first call on that GPU until the process ends; larger requests fail with
 * EINVAL before anything is launched.  Every call on one GPU shares that
 * array: calls that overlap in time on the same GPU (from several threads
 * or streams) race and must be serialised by the caller.  Runs on the
 * factor's stream and returns after it completes. */
rsd_status rsd_matvec_noalloc(rsd_factor* f, const double* x, int64_t nrhs, double* y);

/* Release a factor and all its device memory.  NULL is a no-op. */
void rsd_free(rsd_factor* f);

/* Description of the last error on this thread ("" if none). */
const char* rsd_last_error(void);

/* ---- inspection --------------------------------------------------------- */

typedef struct rsd_factor_stats {
    int64_t n_points, nx, ny;
    int32_t n_levels;        /* tree levels including the root               */
    int32_t n_boxes;
    int32_t layers;          /* m actually used                              */
    int32_t precision;
    int64_t factor_bytes;    /* device bytes held by the factor              */
    double factor_flops;     /* algorithmic flops of the build (model)       */
    double solve_bytes;      /* factor bytes streamed by one solve           */
    double build_ms;         /* device time of the last build                */
    int32_t complex_values;  /* 1: Helmholtz factor; right-hand sides and
                                solutions are interleaved complex (c128)      */
    int32_t solve_graphs;    /* solve widths whose sweeps replay a captured
                                graph (RSD_FLAG_SOLVE_GRAPH)                  */
} rsd_factor_stats;

rsd_status rsd_factor_get_stats(const rsd_factor* f, rsd_factor_stats* out);

/* Per-box description: level (height above the leaves, 0 = leaves), grid
 * origin/size, skeleton size k and residual size r. */
typedef struct rsd_box_info {
    int32_t level, x0, y0, ax, ay, k, r, parent;
} rsd_box_info;
rsd_status rsd_factor_box_info(const rsd_factor* f, int32_t box, rsd_box_info* out);

/* Truncation record of the interpolation T of a box's type (Sec. 2.1: the
 * interpolative decomposition keeps the leading columns of the column-pivoted
 * QR whose |R_jj| exceeds tol |R_11|).  n_problems is 0 when the type has no
 * interpolation (the root), 1 when its problem was solved whole, and 2 or 4
 * when it was split into mirror-symmetry sectors; rank[s] is the number of
 * columns kept in problem s and scale[s] its |R_11| reference.  The sectors
 * of one type share one reference: the largest column norm over all of
 * them, which is the first pivot of the whole problem in the sector basis.
 * Unused entries are zero.  A damped problem keeps every column (rank = k);
 * problems too large for the damping rows in the panel kernel's local
 * memory fall back to truncation (damped = 0).  Waits for the factor's
 * stream; call it when no solve is running on the factor.  Errors: RSD_EINVAL (null argument, box
 * out of range). */
typedef struct rsd_interp_info {
    int32_t n_problems;
    int32_t rank[4];
    double scale[4];
    int32_t damped;        /* 1: solved as damped least squares (RSD_FLAG_NO_DAMPING) */
} rsd_interp_info;
rsd_status rsd_factor_interp_info(const rsd_factor* f, int32_t box, rsd_interp_info* out);

/* Copy one per-box block to host memory (column-major):
 *   which = 0: T_i (k x r), the interpolation of Sec. 3.1 (R_i = [I T_i])
 *   which = 1: E_i (k x k), needs RSD_FLAG_KEEP_E
 *   which = 2: active point ids of the box in [skeleton; residual] order
 *              (k + r int64 grid indices i * ny + j), independent of dtype.
 * dst must hold the block; elements are double (complex: interleaved). */
rsd_status rsd_factor_get_block(const rsd_factor* f, int32_t box, int32_t which, void* dst);

/* ---- device memory cache -------------------------------------------------
 *
 * Device buffers of builds, factors and solves come from a per-device cache:
 * a freed buffer is kept and handed out again to a later request of about
 * the same size (blocks are classed by size: powers of two up to 1 MiB, then
 * 2 MiB multiples; a cached block at most 1/8 larger than the request is
 * reused), so repeated builds do not pay hipMalloc / hipFree for their
 * arenas.  A block enters the cache only after its last use has completed.
 * At most `limit` bytes stay cached per device (default: the smaller of
 * 16 GiB and 1/8 of the device memory); an allocation that fails first hands
 * the device's cache back to HIP and tries again.  Thread-safe. */

/* Hand every cached block of `device` (< 0: of every device) back to HIP. */
rsd_status rsd_pool_trim(int32_t device);

/* Set the per-device cache limit in bytes (< 0: back to the default);
 * blocks beyond a smaller limit are handed back at once. */
rsd_status rsd_pool_set_limit(int64_t bytes);

/* Bytes currently cached (idle) for `device` (< 0: all devices). */
rsd_status rsd_pool_cached_bytes(int32_t device, int64_t* out);

/* ---- kernel timing -------------------------------------------------------- */

/* Kernel classes timed by the built-in profiler. */
typedef enum rsd_prof_class {
    RSD_PROF_FACTOR_GEMM_F64 = 0,  /* block updates of the build, float64 MFMA    */
    RSD_PROF_FACTOR_GEMM_F32 = 1,  /* block updates of the build, float32 MFMA    */
    RSD_PROF_INTERP = 2,           /* proxy matrices + pivoted QR for T           */
    RSD_PROF_GJ_PIVOT = 3,         /* Gauss-Jordan pivot-block steps              */
    RSD_PROF_ASSEMBLY = 4,         /* leaf blocks, parent assembly, transposes    */
    RSD_PROF_SOLVE_GEMM = 5,       /* level sweeps of the inverse apply           */
    RSD_PROF_SOLVE_MOVE = 6,       /* gathers/scatters between levels             */
    RSD_PROF_MATVEC = 7,           /* exact float64 residual products             */
    RSD_PROF_NCLASS = 8
} rsd_prof_class;

/* Enable (on != 0) or disable the profiler and clear its records.  While
 * enabled, every launch of a timed class is bracketed by HIP events on the
 * stream it runs on (the GEMM launches carry theirs in the dispatch, so they
 * time the kernel alone; the other classes record marker events around their
 * launches); totals are read with rsd_profile_query.  The profiler is
 * process-wide; records from several threads are collected under a lock, but
 * enabling or querying while other threads launch work is not supported. */
rsd_status rsd_profile_enable(int32_t on);

/* As rsd_profile_enable, but only the classes whose bit (1 << cls) is set in
 * `mask` are bracketed (0 disables).  Events are reused across enables, so a
 * run that enables the same classes twice creates no events the second
 * time. */
rsd_status rsd_profile_enable_mask(uint32_t mask);

/* Pause (paused != 0) or resume an enabled profiler without clearing its
 * records: while paused no launch is bracketed, so a caller can time a
 * sample of its steps and run the others without events.  Enabling clears
 * the pause.  Like enabling, not to be called while other threads launch
 * work. */
rsd_status rsd_profile_pause(int32_t paused);

/* Totals for one class since the last enable: summed device time of its
 * launches (ms), launch count, algorithmic flops and algorithmic bytes
 * (operands read + written once) of those launches.  Synchronises the
 * device. */
rsd_status rsd_profile_query(int32_t cls, double* total_ms, int64_t* launches,
                             double* flops, double* bytes);

/* Launches recorded since the last enable, in the order they were enqueued
 * (per thread).  Record i: class, device time (ms), algorithmic flops and
 * bytes, and work-groups launched (0 where not recorded).  Synchronises on
 * that launch. */
rsd_status rsd_profile_record_count(int64_t* n);
rsd_status rsd_profile_record(int64_t i, int32_t* cls, double* ms, double* flops, double* bytes,
                              int64_t* groups);

/* ---- serving: resident factors, queued solves ------------------------------
 *
 * A server keeps factors resident in device memory and answers solve
 * requests (Algorithm 6 applied to queued right-hand sides) from worker
 * threads; factor requests are built by a builder thread of its own, so a
 * build overlaps on the device with the solves of resident factors.
 * Requests for one factor that are waiting together are coalesced into one
 * multi-RHS solve (padded to a power of two of columns, so each factor keeps
 * at most seven solve plans); different factors are served concurrently,
 * each on its own stream.
 *
 * Admission is by memory and slots, continuously: a factor request is
 * queued (first come, first served) and admitted when its device bytes
 * (rsd_estimate_factor_bytes plus the coalescing and solve vectors of a full
 * batch, 6 N max_coalesce doubles) fit in the budget beside the resident
 * factors and a slot is free.  With evict_idle = 1 the least recently used
 * idle factors (no queued or running solves) are evicted to make room; with
 * evict_idle = 0 the request waits until factors are released.  A request
 * larger than the whole budget fails at once with ENOMEM.  Solves may be
 * submitted for a factor that is still queued or building; they run once it
 * is resident (or complete with the build's error status).
 * Latency = submission to completion (host clock). */
typedef struct rsd_server rsd_server;

typedef struct rsd_server_options {
    int64_t mem_budget;    /* device bytes for resident factors; 0 => 3/4 of free */
    int32_t max_slots;     /* resident factors at most; 0 => 16                */
    int32_t n_workers;     /* solve threads; 0 => 2                            */
    int32_t max_coalesce;  /* right-hand sides per coalesced solve; 0 => 64    */
    int32_t device;        /* HIP device; < 0 => the current device            */
    int32_t evict_idle;    /* 1 => evict idle factors (LRU) to admit new ones;
                              0 => queue factor requests until memory frees    */
} rsd_server_options;

typedef struct rsd_server_stats {
    int64_t n_requests;    /* solve requests submitted                        */
    int64_t n_done;        /* completed (any status)                          */
    int64_t n_batches;     /* coalesced solves run                            */
    int64_t n_factors;     /* resident factors (built and admitted)           */
    int64_t n_evicted;     /* factors evicted for admission                   */
    int64_t resident_bytes;/* bytes of resident and building factors          */
    double p50_ms, p99_ms; /* request latency percentiles                     */
    double mean_batch_rhs; /* right-hand sides per coalesced solve (unpadded) */
    double rhs_per_s;      /* completed right-hand sides / seconds since the
                              first submission                                 */
    int64_t n_queued_factors; /* factor requests waiting for admission or
                                 being built                                   */
    int64_t n_built;       /* factor builds completed (any status)            */
} rsd_server_stats;

/* opt NULL => defaults.  Starts the worker threads and the builder thread. */
rsd_status rsd_server_create(const rsd_server_options* opt, rsd_server** out);
/* Queues a factor request (as rsd_build_factor, Sec. 2.4 / Algorithm 1;
 * opt->hip_stream must be NULL: the server gives each factor its own
 * stream).  points, a (and kernel->contrast_b) are copied before the call
 * returns (host or device pointers); the grid is checked at once (ENOTGRID,
 * EINVAL).  *factor_id receives its handle for submit_solve and
 * wait_factor.  ENOMEM at once when the factor alone exceeds the budget;
 * otherwise the request waits for admission (see above). */
rsd_status rsd_server_submit_factor(rsd_server* s, const double* points, int64_t n_points,
                                    const rsd_kernel* kernel, const double* a, double tol,
                                    const rsd_options* opt, int64_t* factor_id);
/* Waits up to timeout_ms (< 0 => forever) until a factor request is built:
 * OK once resident, the build's status if it failed, EAGAIN on timeout,
 * EINVAL for an unknown or released id. */
rsd_status rsd_server_wait_factor(rsd_server* s, int64_t factor_id, int32_t timeout_ms);
/* Releases a factor (resident, or still queued); EAGAIN while it is being
 * built or has queued or running solves, EINVAL for an unknown id. */
rsd_status rsd_server_release_factor(rsd_server* s, int64_t factor_id);
/* Queues x = A^{-1} rhs (N x nrhs column-major, host or device pointers).
 * Both buffers are borrowed until the request completes (rsd_server_wait).
 * *ticket identifies the request.  EINVAL for an unknown factor or nrhs
 * above max_coalesce. */
rsd_status rsd_server_submit_solve(rsd_server* s, int64_t factor_id, const double* rhs,
                                   int64_t nrhs, double* x, int64_t* ticket);
/* Waits up to timeout_ms (< 0 => forever) for a request; returns its status
 * (OK, ENOCONV, ...) and info, and forgets the ticket; EAGAIN on timeout
 * (the ticket stays valid); EINVAL for an unknown ticket. */
rsd_status rsd_server_wait(rsd_server* s, int64_t ticket, int32_t timeout_ms, rsd_solve_info* info);
/* 1 when the request has completed, 0 while pending, -1 for an unknown ticket. */
int32_t rsd_server_poll(rsd_server* s, int64_t ticket);
rsd_status rsd_server_get_stats(rsd_server* s, rsd_server_stats* out);
/* Finishes the queued requests (builds included), stops the threads and
 * frees every factor. */
void rsd_server_destroy(rsd_server* s);

/* ---- dense building blocks ------------------------------------------------ */

/* C = alpha op(A) op(B) + beta C with the library's MFMA grouped-GEMM kernel
 * (one product).  dtype 0 = float64, 1 = float32.  Column-major; op = transpose
 * when tA / tB is 1.  Pointers host or device; the call is synchronous. */
rsd_status rsd_gemm(int32_t dtype, int32_t M, int32_t N, int32_t K, int32_t tA, int32_t tB,
                    double alpha, const void* A, int32_t lda, const void* B, int32_t ldb,
                    double beta, void* C, int32_t ldc);

/* In-place inverse of an n x n matrix by the library's blocked Gauss-Jordan
 * elimination in natural order (no row exchanges: for symmetric positive
 * definite or diagonally dominant matrices, the blocks the solver inverts).
 * dtype bit 0: float32 (else float64); bit 1: paired pivots, the form used
 * for complex factors (n even; rows and columns 2i, 2i + 1 hold the real
 * form [[re, im], [im, -re]] of a complex entry, and each step eliminates
 * such a pair with its 2 x 2 inverse).  Returns ESINGULAR when a pivot
 * (pair) is singular. */
rsd_status rsd_gj_invert(int32_t dtype, int32_t n, void* A, int32_t lda);

/* ---- host-only planning (no device needed) ------------------------------ */

/* Integral of the kernel over the square cell of side h centred on its
 * point, the diagonal term of the Nystrom matrix (Sec. 5; k the wavenumber
 * of the Helmholtz kernel (i/4) H0^(1)(k r) of Sec. 5.3, ignored for
 * Laplace).  Host only. */
rsd_status rsd_self_cell_integral(int32_t kernel_type, double h, double k, double* re, double* im);
/* Device bytes of the factor rsd_build_factor would keep for an nx x ny grid
 * with this kernel (NULL => Laplace) and these options (the per-box
 * (k + r)^2 blocks of Algorithm 1 in the Schur form and the interpolation
 * blocks, four times the entries for the complex Helmholtz kernel): equal to
 * rsd_factor_stats.factor_bytes of a factor built with every box's blocks
 * (a varying a, or RSD_FLAG_NO_DEDUP), an upper bound for one that shares
 * them (constant a).  Interface skeleton points (interface_ppw) are placed
 * for the grid spacing 1 / max(nx, ny) of the unit square.  Host only. */
rsd_status rsd_estimate_factor_bytes(int64_t nx, int64_t ny, const rsd_kernel* kernel, double tol,
                                     const rsd_options* opt, int64_t* bytes);
/* Number of boxes and levels the tree of Sec. 2.2 / Sec. 3.1 produces for an
 * nx x ny grid, and per-box sizes.  Pure host computation, usable without a
 * GPU; boxes are numbered level by level from the leaves.  interface_step:
 * spacing in grid cells of the interface skeleton points (see
 * rsd_options.interface_ppw), 0 for none. */
typedef struct rsd_plan rsd_plan;
rsd_status rsd_plan_create(int64_t nx, int64_t ny, int32_t leaf_side, int32_t layers,
                           int32_t interface_step, rsd_plan** out);
int32_t rsd_plan_n_boxes(const rsd_plan* p);
int32_t rsd_plan_n_levels(const rsd_plan* p);
rsd_status rsd_plan_box_info(const rsd_plan* p, int32_t box, rsd_box_info* out);
/* active point ids of a box, [skeleton; residual] order (k + r int64) */
rsd_status rsd_plan_box_points(const rsd_plan* p, int32_t box, int64_t* dst);
/* Mirror reflections of the box (u -> ax-1-u along an even side ax, v ->
 * ay-1-v along an even side ay) that map its skeleton, residual and proxy
 * sets onto themselves: *group = bit 0 the u reflection, bit 1 the v
 * reflection (0: none, or a box without an interpolation problem).  The
 * factorization splits such a box type's least-squares problem into 2 or 4
 * sector problems. */
rsd_status rsd_plan_box_symmetry(const rsd_plan* p, int32_t box, int32_t* group);
/* The sector problems the interpolation of a plan is solved as (Sec. 3.1;
 * the truncated pivoted QR of Sec. 2.1 per problem), one entry per problem in
 * the order a chain of all the plan's box types lists them: 7 int32 per entry
 *   owner  index of the box type's interpolation problem in the plan
 *   sec    symmetry character solved (0..3), or -1 when solved whole
 *   g0,gn  the sector group: list index of its first problem, and its size
 *          (1, 2 or 4); the truncation scale |R11| of every problem is the
 *          largest column norm over exactly [g0, g0 + gn)
 *   p,k,r  rows, skeleton and residual columns of the (sector) problem
 * split = 0 lists every problem whole.  table NULL => only *n_problems is set.
 * The table is checked as rsd_check_interp_groups does before it is returned.
 * Host only. */
rsd_status rsd_plan_interp_groups(const rsd_plan* p, int32_t split, int32_t* n_problems,
                                  int32_t* table);
/* Checks a table in that format: every group lies inside the list, contains
 * its problem and is made of consecutive sectors of one owner with the
 * characters of one reflection group.  EINVAL (message names the entry) if
 * not.  Host only; the build runs the same check before its kernels read the
 * groups. */
rsd_status rsd_check_interp_groups(int32_t n_problems, const int32_t* table);
void rsd_plan_free(rsd_plan* p);

/* Grid detection used by rsd_build_factor: on success nx, ny, h and perm
 * (perm[g] = caller index of grid point g = i * ny + j) are filled. */
rsd_status rsd_detect_grid(const double* points_host, int64_t n_points,
                           int64_t* nx, int64_t* ny, double* h, int64_t* perm);

#ifdef __cplusplus
}
#endif

#endif /* RSD_H */
