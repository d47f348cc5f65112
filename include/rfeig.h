/*
 * rfeig -- composite-rule rational-filter interior eigensolver, MI355X (gfx950).
 *
 * C ABI of the library.  It finds every eigenpair (lambda, x) of a sparse
 * non-Hermitian pencil A x = lambda B x with lambda inside the disk
 * D = { z : |z - c| < r }  (Chen & Li, "Interior Eigensolver Based on
 * Rational Filter with Composite Rule", Sec. 1, eq. problem), by subspace
 * iteration with the composite-rule trapezoidal filter R_{c,r,pq}(B^{-1}A)
 * (Sec. 3.2, Alg. composite).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are interleaved (re, im) pairs of IEEE doubles
 *   (complex128).  Blocks of vectors are column-major with a leading
 *   dimension >= n.
 * - Sparse matrices are CSR in HOST memory (int32 row pointers and column
 *   indices, complex128 values).  The library copies them at plan creation;
 *   the caller may free them afterwards.
 * - Block arguments (Y, U, X, Z) are DEVICE pointers owned by the caller.
 *   Scalar outputs (eigenvalues, errors, flags, counters) are HOST arrays
 *   owned by the caller.
 * - Every call enqueues its GPU work on the stream given at plan creation and
 *   returns after that stream has drained, so outputs are ready on return.
 * - Errors are returned as rf_status; no call aborts or throws across the
 *   ABI.  rf_last_error() gives a message for the plan's last failure.
 *   RF_ERR_DEVICE leaves the plan unusable (destroy it).
 * - One plan must not be used from two host threads at once.
 */
#ifndef RFEIG_H
#define RFEIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RF_OK = 0,
    RF_ERR_ARG = 1,       /* bad argument: sizes, NULL pointers, r <= 0, p or q < 1, w < 1 or w > n */
    RF_ERR_NOMEM = 2,     /* device allocation failed */
    RF_ERR_SINGULAR = 3,  /* exact zero pivot: a pole lies on an eigenvalue */
    RF_ERR_NOCONV = 4,    /* iteration cap reached; partial results are returned and flagged */
    RF_ERR_DEVICE = 5,    /* a HIP call failed; the plan is unusable */
    RF_ERR_STATE = 6      /* call out of order (e.g. filter before factor_shifts) */
} rf_status;

/* Sparse square matrix in CSR form, host memory.  val holds 2*nnz doubles. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *rowptr;   /* n + 1 entries */
    const int32_t *colind;   /* nnz entries, 0-based */
    const double *val;       /* nnz complex values, interleaved re/im */
} rf_csr;

/* Solver options.  Fill with rf_default_opts() and then set the disk. */
typedef struct {
    double c_re, c_im;       /* disk centre c */
    double r;                /* disk radius r > 0 */
    int32_t p;               /* inner trapezoidal nodes k1: factorized poles (eq. pwtp) */
    int32_t q;               /* outer trapezoidal nodes k2: multi-shift GMRES shifts (Thm. Rcrm) */
    int32_t w;               /* block width n_col of the subspace iteration */
    double sigma_re, sigma_im; /* HSRR shift sigma; NaN in sigma_re means sigma = c (Sec. 6) */
    double tau;              /* target relative error of converged pairs (eq. rel-error); default 1e-10 */
    double tau_g;            /* ghost threshold tau_g (Sec. 3.2); default 1e-2 */
    double gmres_tol;        /* outer-solve tolerance, relative per column and shift; default 1e-12 */
    int32_t max_subspace_it; /* cap on subspace iterations; default 10 (Sec. 6.3) */
    int32_t max_krylov_blocks; /* cap on block-Arnoldi steps per filter application; default 150 */
    int32_t subblock;        /* Krylov sub-block width b dividing w (0 = automatic) */
    int32_t expected_count;  /* expected eigenvalue count s inside D, -1 if unknown */
    int32_t tile;            /* band tile size nb: 16, 32, 64, 128 or 256, >= the bandwidth (0 = automatic: the smallest such) */
    int32_t trsm_cols;       /* right-hand sides per band-solve workgroup: 1, 2 or 4 (0 = automatic, 3 and 5..8 act as 4) */
    uint64_t seed;           /* seed of the start block when none is given */
    int32_t q_max;           /* largest outer node count of rf_solve_region_adaptive (0 = q) */
    int32_t precision;       /* 0: complex128 band solves; 1: precision form -- complex64 copies of the
                                (complex128) factors for every band solve, the outer GMRES to
                                max(gmres_tol, 1e-6), and from the second sweep of rf_solve_region on
                                the filter applied through the complex128 residual of the Ritz pairs */
    int32_t refine;          /* precision form: FP64 iterative-refinement steps of every shifted solve
                                K_i x = b (0..4): r = b - K_i x in complex128 from the sparse A and B,
                                x += K_i^{-1} r with the complex64 factors; 0 with precision 0 */
    int32_t no_graph;        /* 0: rf_factor_shifts records its fixed launch sequence once in a HIP
                                graph (on a non-null stream) and replays it; 1: plain launches */
    int32_t solve_form;      /* complex128 band solves of eq. linearsolve2: 0 (automatic) = the
                                cluster form wherever it applies (tile 64 or 128, precision 0,
                                not an adjoint plan): the factorization also stores the products
                                L21 Linv, Uinv Linv, Uinv U1, Uinv U2 of every block (4/5 of the
                                factor storage again) and each solve runs clusters of nb/16
                                workgroups per pole and 16 right-hand sides on the FP64 matrix
                                cores; 1 = the per-slice form only (no product storage) */
} rf_opts;

/* Per-call statistics of a filter application. */
typedef struct {
    int32_t krylov_steps;    /* block-Arnoldi steps taken (applications of G to the basis) */
    int32_t converged;       /* 1 if every column met gmres_tol for every shift */
    double max_residual;     /* largest relative residual over shifts and columns */
    int64_t inner_columns;   /* vectors G was applied to (each costs p solve pairs) */
    double ms_total;         /* wall time of the call */
} rf_filter_info;

/* Output of rf_solve_region.  All arrays are caller-owned.
 * Slots 0..count-1 hold the converged pairs inside D (|lambda - c| < r,
 * e <= tau); the remaining w - count slots hold the other Ritz pairs of the
 * last sweep, with flags telling inside / filtered / converged. */
typedef struct {
    double *lambda;          /* host, 2*w doubles (complex) */
    void *X;                 /* device, n x w complex128, leading dimension ldx; unit 2-norm columns */
    int64_t ldx;
    double *err;             /* host, w relative errors e_i (eq. rel-error) */
    int32_t *flags;          /* host, w: bit0 inside D, bit1 e < tau_g, bit2 e <= tau */
    int32_t count;           /* out: converged pairs inside D */
    int32_t sweeps;          /* out: subspace iterations used */
    int32_t converged;       /* out: 1 if the stopping rule of Alg. composite was met */
    int32_t krylov_steps[16];/* out: block-Arnoldi steps per sweep (first 16 sweeps) */
    double ms_filter;        /* out: time in filter applications */
    double ms_hsrr;          /* out: time in projection, QZ and error evaluation */
} rf_result;

typedef struct rf_plan *rf_plan_t;

/* Device-memory callbacks through which a plan or batch obtains ALL of its device
 * memory: band factors, Krylov basis, work and scratch buffers (the storage that the
 * pre-factorization loop and the filter of Alg. composite need besides the caller's
 * blocks).  A caller that manages device memory itself (e.g. PyTorch's caching
 * allocator) passes its own; NULL selects hipMalloc / hipFree.
 *   alloc(bytes, ctx): device memory of at least `bytes` bytes on the current device,
 *       aligned to at least 16 bytes, or NULL on failure (the call then returns
 *       RF_ERR_NOMEM).  Called only inside rf_plan_create / rf_batch_create /
 *       rf_plan_create_adjoint, from the calling thread.
 *   free(ptr, ctx): returns one pointer obtained from alloc.  Called only inside
 *       rf_plan_destroy / rf_batch_destroy (and on creation failure), from the calling
 *       thread, after the plan's streams have drained, so the memory may be reused
 *       at once.
 * The struct is copied; the callbacks and ctx must stay valid until the plan (or
 * batch) is destroyed.  Pinned host staging buffers are not routed through it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} rf_allocator;

/* Defaults: p = 4, q = 8, w = 32, tau = 1e-10, tau_g = 1e-2, gmres_tol = 1e-12,
 * max_subspace_it = 10, max_krylov_blocks = 150, sigma = c, seed = 0, q_max = 0. */
void rf_default_opts(rf_opts *opts);

/* Copy the pencil to the device, compute the trapezoidal poles/weights of the
 * inner rule (eq. pwtp, Sec. 2.2) and the outer shifts/weights (Thm. Rcrm,
 * Sec. 5), size the band tiles from the band extents of pattern(A) and
 * pattern(B), and allocate every device buffer the plan will use, through
 * `allocator` (NULL = hipMalloc).  hip_stream: a hipStream_t (NULL = the null
 * stream).  On failure *out may still be set: read rf_last_error, then destroy it. */
rf_status rf_plan_create(const rf_csr *A, const rf_csr *B, const rf_opts *opts,
                         const rf_allocator *allocator, void *hip_stream, rf_plan_t *out);

/* Band LU with partial pivoting of K_i = p_i B - A for the p inner poles
 * (Alg. composite, the pre-factorization loop).  RF_ERR_SINGULAR on an exact
 * zero pivot. */
rf_status rf_factor_shifts(rf_plan_t plan);

/* Z = G(X) = sum_i w_i K_i^{-1} B X  (eq. linearsolve2), ncols <= w columns.
 * X and Z are device blocks (n x ncols); they may not overlap. */
rf_status rf_apply_inner(rf_plan_t plan, const void *X, int64_t ldx, int32_t ncols,
                         void *Z, int64_t ldz);

/* rf_apply_inner for callers that cannot allocate device memory or synchronize
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, but the work blocks (per-pole forward results and
 * solutions, the B X staging) live in one file-scope device array of the library,
 * 64 MiB per device, held from the first call on a device until the process ends;
 * the call allocates nothing and only enqueues its work on the plan stream (no stream
 * synchronization: Z is ready when the stream reaches that point).  Columns are
 * processed in chunks that fit the array; ncols may exceed w.  RF_ERR_ARG if a single
 * column does not fit (n_pad (p (16 or 8) + 16 + 16) bytes, n_pad = n rounded up to
 * the tile).  All calls on one device share the array: calls that can overlap on one
 * device (different streams, different plans, different threads) race; order them. */
rf_status rf_apply_inner_noalloc(rf_plan_t plan, const void *X, int64_t ldx, int32_t ncols,
                                 void *Z, int64_t ldz);

/* U = R_{c,r,pq}(B^{-1}A) Y = sum_j c'_j (G - s_j I)^{-1} G(Y)   (eq. linearsolve1abs)
 * by block multi-shift GMRES on one shared Krylov basis.  The sign of c'_j is
 * the one for which the sum equals +R_{c,r,pq} (the proof of Thm. Rcrm).
 * ncols must equal the plan's w.  info may be NULL.  RF_ERR_ARG if an entry of Y
 * is not finite; RF_ERR_NOCONV (U still written, info->converged = 0) if a column
 * misses gmres_tol within max_krylov_blocks steps. */
rf_status rf_filter_apply(rf_plan_t plan, const void *Y, int64_t ldy, int32_t ncols,
                          void *U, int64_t ldu, rf_filter_info *info);

/* Alg. composite: subspace iteration with the composite filter and HSRR
 * (Sec. 2.1) until the filtered count is stable and every filtered error is
 * <= tau.  Y0: device n x w start block (NULL = seeded Gaussian; RF_ERR_ARG if an
 * entry is not finite).  Calls rf_factor_shifts first if it has not run.
 * RF_ERR_NOCONV if the sweep cap is reached (results still filled in). */
rf_status rf_solve_region(rf_plan_t plan, const void *Y0, int64_t ldy, rf_result *res);

/* Alg. composite2 (Sec. 3.2): the composite filter without subspace iteration.
 * Y0 (device n x w, NULL = seeded Gaussian) is orthonormalised once and
 * Ytilde = G(Y0) is formed once; then for k2 = q, 2q, 4q, ... <= q_max the outer
 * solves (G - s_j I) U_j = Ytilde are solved for ALL k2 shifts on the one shared,
 * growing Krylov basis (the shifts of 2 k2 nodes do not contain those of k2, so
 * none are reused), U = sum_j c'_j U_j = R_{c,r,p k2}(B^{-1}A) Y0, and HSRR with the
 * ghost test runs on U; the loop stops when the filtered count repeats (or equals
 * expected_count at the first level) and every filtered error is <= tau.
 * res->sweeps = levels used, res->krylov_steps[t] = basis depth at level t.
 * q_max of the plan must be >= q (the plan sizes the per-shift storage by it).
 * RF_ERR_NOCONV when q_max is reached first (results still filled in). */
rf_status rf_solve_region_adaptive(rf_plan_t plan, const void *Y0, int64_t ldy, rf_result *res);

/* Timing of the band kernels, for roofline accounting.  Times are summed
 * HIP-event intervals recorded on the plan stream around each launch. */
typedef struct {
    int64_t solve_launches;  /* launches of the multi-RHS band-solve kernel */
    int64_t solve_columns;   /* right-hand sides summed over those launches (each solved for all p poles) */
    double solve_ms;         /* summed duration of those launches */
    int64_t factor_launches; /* launches of the band-factorization kernel pair */
    double factor_ms;        /* summed duration (factorization + triangle inversion) */
} rf_kernel_stats;

/* on != 0: reset the counters and start timing; on == 0: stop. */
rf_status rf_profile_enable(rf_plan_t plan, int32_t on);

/* Copy the counters accumulated since rf_profile_enable(plan, 1); synchronizes
 * the plan stream. */
rf_status rf_profile_read(rf_plan_t plan, rf_kernel_stats *out);

/* Generalized eigenvalues and right eigenvectors of a small dense pencil (A, B),
 * the "qz" step of HSRR (Sec. 2.1): complex QZ to the generalized Schur form,
 * then back-substitution on the triangular pencil and back-transformation.
 * Host memory: A, B are n x n column-major complex128 (2 n^2 doubles each, not
 * modified); alpha, beta get n complex values with lambda_i = alpha_i / beta_i;
 * vr gets n unit-2-norm eigenvectors (columns, n x n complex128).  Runs on the
 * CPU only.  Returns 0, or -1 if the QZ iteration did not converge. */
int rf_dense_eig(int32_t n, const double *A, const double *B, double *alpha, double *beta,
                 double *vr);

/* rf_solve_region on `count` distinct plans at once, each on a host thread of its own
 * and its plan's stream (plans created on different streams run concurrently on the
 * device; plans sharing a stream still give the right results); factor != 0 runs
 * rf_factor_shifts first on every plan (concurrently too).  When adjoint plans are in
 * the list, the plans that own factors are factorized first (where factor != 0 or
 * they have no factors yet), then the adjoint plans take their transposes, then all
 * plans are solved concurrently.  Y0, ldy: host arrays
 * of start blocks and leading dimensions (NULL or NULL entries: seeded Gaussian); res,
 * status: host arrays of count results and return codes.  Returns RF_OK if every plan
 * returned RF_OK, else the first other code in plan order; RF_ERR_ARG if a plan
 * appears twice.  For independent problems, e.g. a pencil and its adjoint. */
rf_status rf_solve_regions(int32_t count, rf_plan_t *plans, int32_t factor, const void *const *Y0,
                           const int64_t *ldy, rf_result *res, rf_status *status);

/* ---------------------------------------------------------------------------
 * Differentiation form.  For a simple eigenvalue lambda of A x = lambda B x with
 * right vector x and left vector y (y^H A = lambda y^H B), first-order
 * perturbation theory (textbook; the paper does not treat it) gives
 *     d lambda = y^H (dA - lambda dB) x / (y^H B x).
 * The left vectors are the right eigenvectors of the adjoint pencil (A^H, B^H) at
 * conj(lambda), which the same solver finds over the mirrored disk D(conj c, r).
 * ------------------------------------------------------------------------- */

/* A new plan for the adjoint pencil (A^H, B^H) with the options of `plan` and the
 * disk centre (and an explicit HSRR shift) conjugated; its trapezoidal poles are the
 * conjugates of the plan's (eq. pwtp, the node angles are symmetric), so its shifted
 * matrices are the K_i^H of `plan`.  It does not factorize: rf_factor_shifts on it
 * (after rf_factor_shifts on `plan`) makes conjugate-transposed copies of `plan`'s band
 * factors and row orders, and its solves are the K_i^H = U_i^H L_i^H P_i^T sweeps over
 * them.  `plan` must stay alive (and keep its factors) while the adjoint plan is used;
 * refactorizing `plan` needs rf_factor_shifts on the adjoint plan again.  Complex128
 * only (precision 0).  Destroyed with rf_plan_destroy.  Errors as rf_plan_create. */
rf_status rf_plan_create_adjoint(rf_plan_t plan, void *hip_stream, rf_plan_t *out);

/* Vector-Jacobian product of eigenvalues with respect to the stored entries of A
 * and B (in the CSR order given at plan creation):
 *     gA[e] = sum_i g_i * d lambda_i / d A[row(e), col(e)]
 *           = sum_i g_i conj(y_i[row]) x_i[col] / (y_i^H B x_i),
 *     gB[e] = -sum_i g_i lambda_i conj(y_i[row]) x_i[col] / (y_i^H B x_i).
 * s (0..w of the plan) right pairs: lambda (host, 2s doubles), X (device n x s, ldx);
 * s_left adjoint pairs from the adjoint plan: mu (host, 2 s_left doubles), Yl (device
 * n x s_left, ldyl).  Each lambda_i is paired with the mu_j whose conjugate is nearest;
 * RF_ERR_ARG if that distance exceeds 1e-6 (|c| + r) or two lambdas pick the same mu,
 * or if y^H B x = 0.  g: host 2s doubles.  gA: device nnz(A) complex128 (written);
 * gB: device nnz(B) complex128 or NULL.  denom (host 2s doubles, optional) gets
 * y_i^H B x_i and pair (host s ints, optional) the chosen j.  Vector scaling is free:
 * the quotient does not depend on the norms of x_i, y_i.  Runs on the plan stream and
 * uses the plan's work buffers. */
rf_status rf_eig_vjp(rf_plan_t plan, int32_t s, const double *lambda, const void *X, int64_t ldx,
                     int32_t s_left, const double *mu, const void *Yl, int64_t ldyl,
                     const double *g, void *gA, void *gB, double *denom, int32_t *pair);

/* ---------------------------------------------------------------------------
 * Batched form: many disks D_d = { |z - c_d| < r_d } of ONE pencil, solved
 * independently (Sec. 1: the solver covers several regions in parallel to build
 * up a partial or full eigen-decomposition).  All disks' poles are factorized
 * together, so the band factorization runs with sum_d p_d independent chains in
 * one launch sequence, and the disks' subspace iterations run concurrently, each
 * on a stream and host thread of its own.
 * ------------------------------------------------------------------------- */
typedef struct rf_batch *rf_batch_t;

/* opts: host array of ndisks option sets, one per disk (its own c, r, p, q, w,
 * tolerances); every entry must give the same tile (0 = automatic).  The device
 * memory is the factor storage of sum_d p_d poles plus each disk's Krylov and
 * HSRR buffers, all obtained through `allocator` (NULL = hipMalloc); the library
 * creates one non-blocking stream per disk and runs
 * the factorization on hip_stream.  On failure *out may still be set: read
 * rf_batch_last_error, then rf_batch_destroy it. */
rf_status rf_batch_create(const rf_csr *A, const rf_csr *B, const rf_opts *opts, int32_t ndisks,
                          const rf_allocator *allocator, void *hip_stream, rf_batch_t *out);

/* Factorize K_i = p_i B - A for every pole of every disk (the disks' step 2 of
 * Alg. composite, batched).  RF_ERR_SINGULAR names the first disk with an exactly
 * singular shifted pencil; then no disk is usable until a later call succeeds. */
rf_status rf_batch_factor(rf_batch_t batch);

/* The plan of disk d (0 <= d < ndisks; NULL if out of range), owned by the batch:
 * every per-plan call works on it (rf_filter_apply, rf_solve_region,
 * rf_solve_region_adaptive, profiling) on the disk's own stream, except
 * rf_factor_shifts, which returns RF_ERR_STATE: its factors come from
 * rf_batch_factor. */
rf_plan_t rf_batch_plan(rf_batch_t batch, int32_t d);

/* Number of disks, or -1. */
int32_t rf_batch_size(rf_batch_t batch);

/* rf_solve_region for every disk, at most `threads` disks at a time (<= 0: all),
 * each on its own host thread and stream.  Y0: host array of ndisks device start
 * blocks (NULL, or a NULL entry: seeded Gaussian), ldy: host array of their leading
 * dimensions (may be NULL when Y0 is); res: host array of ndisks rf_result, filled
 * as by rf_solve_region; status: host array of ndisks per-disk return codes.
 * Returns RF_OK if every disk returned RF_OK, else the code of the first disk that
 * did not (its message in rf_batch_last_error).  Start blocks written on another
 * stream must be complete before the call. */
rf_status rf_batch_solve(rf_batch_t batch, const void *const *Y0, const int64_t *ldy,
                         rf_result *res, rf_status *status, int32_t threads);

/* Bytes of device memory the batch holds (factor storage and every disk plan). */
int64_t rf_batch_device_bytes(rf_batch_t batch);

const char *rf_batch_last_error(rf_batch_t batch);
void rf_batch_destroy(rf_batch_t batch);

/* Problem size n of a plan, or -1. */
int64_t rf_plan_n(rf_plan_t plan);

/* Bytes of device memory the plan holds. */
int64_t rf_plan_device_bytes(rf_plan_t plan);

void rf_plan_destroy(rf_plan_t plan);
const char *rf_status_str(rf_status s);
const char *rf_last_error(rf_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* RFEIG_H */
