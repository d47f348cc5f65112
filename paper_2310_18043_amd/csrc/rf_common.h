// Internal declarations shared by the rfeig host code and kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "rfeig.h"

// ---------------------------------------------------------------------------
// complex FP64 helpers (interleaved re/im in a double2)
// ---------------------------------------------------------------------------
typedef double2 zd;
typedef float2 zf;   // complex64 (single-precision factor tiles)

__host__ __device__ inline zd zmake(double re, double im) { zd r; r.x = re; r.y = im; return r; }
__host__ __device__ inline zd zadd(zd a, zd b) { return zmake(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zd zsub(zd a, zd b) { return zmake(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zd zmul(zd a, zd b) { return zmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline zd zconj(zd a) { return zmake(a.x, -a.y); }
__host__ __device__ inline zd zscale(zd a, double s) { return zmake(a.x * s, a.y * s); }
__host__ __device__ inline double zabs2(zd a) { return a.x * a.x + a.y * a.y; }
// acc += a * b
__host__ __device__ inline void zfma(zd &acc, zd a, zd b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc -= a * b
__host__ __device__ inline void zfms(zd &acc, zd a, zd b) {
    acc.x = fma(-a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
// acc += conj(a) * b
__host__ __device__ inline void zfma_c(zd &acc, zd a, zd b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
__host__ __device__ inline zd zdiv(zd a, zd b) {
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        double t = b.y / b.x, d = b.x + b.y * t;
        return zmake((a.x + a.y * t) / d, (a.y - a.x * t) / d);
    } else {
        double t = b.x / b.y, d = b.x * t + b.y;
        return zmake((a.x * t + a.y) / d, (a.y * t - a.x) / d);
    }
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct DevCsr {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t *rowptr = nullptr;
    int32_t *colind = nullptr;
    zd *val = nullptr;
    bool diagonal = false;     // only diagonal entries (then dval holds them)
    zd *dval = nullptr;        // n entries when diagonal
};

struct HostCsr {               // host copy of a pencil matrix as given (for the adjoint pencil)
    int32_t n = 0;
    std::vector<int32_t> rowptr, colind;
    std::vector<double> val;   // 2 * nnz (interleaved complex)
};

struct BandFactors {
    int nb = 0;                // tile size (>= kl, ku)
    int nblk = 0;              // number of row/column blocks
    int64_t tile_elems = 0;    // nb * nb
    // per pole, per block k: tiles stored back to back, see rf_band.hip
    zd *tiles = nullptr;       // p * nblk * 5 * nb*nb
    int32_t *perm = nullptr;   // p * nblk * 2nb
    zd *window = nullptr;      // p * 2 * (2nb x 3nb) factorization scratch (double-buffered)
    zd *rows = nullptr;        // p * nblk * (nb x 3nb): row blocks of p_i B - A, dense
    int32_t *subperm = nullptr; // p * 2nb: row order of the current sub-panel
    int32_t *info = nullptr;   // p ints: 0 or (1 + first zero-pivot column)
    zf *tiles32 = nullptr;     // complex64 copy of tiles (precision form), or null
    // cluster solve (rf_cluster.hip): fused tiles M, W, V1, V2 per pole and block
    // (p * nblk * 4 * nb*nb, or a batch owner's), the exchange area, the sequence flags
    // and the error words {epoch of a timed-out wait, epoch of a misplaced workgroup}
    zd *ftiles = nullptr;
    zd *xchg = nullptr;
    unsigned long long *cflags = nullptr;
    unsigned *cerr = nullptr;
    unsigned *ctickets = nullptr;  // per-XCD arrival counters (8 x 32 words)
    mutable unsigned cepoch = 0;   // epoch of the last cluster launch
    unsigned cerr_seen = 0;        // launches up to this epoch have been checked
    bool cluster_ok = true;        // false after a reported failure: per-slice solves
    bool adjoint = false;      // tiles hold the conjugate transposes of another plan's
                               // factors (adjoint pencil): solves run the K^H sweeps
    bool ready = false;
};

// HIP-event timing of the band kernels (enabled by rf_profile_enable)
struct KernelProfile {
    bool on = false;
    std::vector<hipEvent_t> pool;          // free events
    struct Pending { hipEvent_t a, b; int64_t cols; int kind; };
    std::vector<Pending> pending;          // recorded, not yet read
    rf_kernel_stats stats{};
    hipEvent_t take();
    void record_begin(hipStream_t s, hipEvent_t &a);
    void record_end(hipStream_t s, hipEvent_t a, int64_t cols, int kind);
    hipError_t drain();                    // sync on the events, fold into stats
    void release();
};

struct rf_plan {
    rf_opts opts;
    mutable KernelProfile prof;
    int64_t n = 0;
    int kl = 0, ku = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int max_lds = 65536;      // dynamic LDS bytes a workgroup may use
    int num_cu = 256;         // compute units of the device
    DevCsr A, B;
    HostCsr hA, hB;
    std::vector<zd> poles, weights;       // inner rule (p)
    std::vector<zd> shifts, oweights;     // outer rule (finite shifts)
    double oextra = 0.0;                  // (1/q) term for odd q
    zd *d_poles = nullptr, *d_weights = nullptr;
    zd *d_shifts = nullptr, *d_oweights = nullptr;
    BandFactors F;
    // work buffers
    zd *rhs = nullptr;        // B X staging: n_pad x w
    zd *ypart = nullptr;      // per-pole forward results: p x n_pad x w
    zd *xpart = nullptr;      // per-pole solutions: p x n_pad x w
    zd *refres = nullptr;     // per-pole refinement residuals: p x n_pad x w (refine > 0)
    // Krylov
    int b = 0, nsub = 0, mmax = 0;
    zd *V = nullptr;          // nsub x (mmax+1) blocks of n x b
    zd *Wk = nullptr;         // n x w
    zd *Gin = nullptr;        // n x w staging of the active basis blocks
    zd *Hm = nullptr;         // nsub x ((mmax+1)b x mmax b) block Hessenberg
    zd *R0 = nullptr;         // nsub x (b x b)
    zd *lsQ = nullptr;        // nq x nsub x mmax x (2b x 2b)
    zd *lsR = nullptr;        // nq x nsub x (mmax b x mmax b)
    zd *lsG = nullptr;        // nq x nsub x ((mmax+1)b x b)
    zd *lsWork = nullptr;     // nq x nsub x ((mmax+1)b x b)
    zd *lsY = nullptr;        // nq x nsub x (mmax b x b)
    zd *ycomb = nullptr;      // nsub x (mmax b x b)
    double *resid = nullptr;  // nq x nsub x b
    double *r0norm = nullptr; // nsub x b column norms of the start block
    zd *ytil = nullptr;       // n x w  G(Y)
    zd *tmp = nullptr;        // n x w  scratch
    double *colnorm = nullptr;// w
    zd *small = nullptr;      // scratch for b x b / w x w matrices
    zd *hbuf = nullptr;       // (mmax+1)b x b Gram-Schmidt coefficients
    zd *rnew = nullptr;       // b x b
    zd *ident = nullptr;      // b x b identity
    zd *partial = nullptr;    // split-N GEMM partials
    int64_t partial_elems = 0;
    int *flag = nullptr;      // device status flags
    int *d_status = nullptr;  // 2w Cholesky breakdown flags (two passes)
    double *d_dratio = nullptr; // 2w Cholesky diagonal ratios
    int *d_active = nullptr;  // w active sub-block indices
    int *h_pinned_int = nullptr; // pinned host mirror of d_active
    char *h_stage = nullptr;     // pinned staging for device-to-host reads
    size_t stage_bytes = 0;
    // HSRR
    zd *hV = nullptr, *hAV = nullptr, *hBV = nullptr, *hW = nullptr, *hX = nullptr;
    zd *hY = nullptr;         // n x w: block being filtered while the host QZ runs
    zd *hV2 = nullptr, *hAV2 = nullptr, *hBV2 = nullptr;  // second basis set (adaptive solver)
    zd *hproj = nullptr;      // 2 * w * w
    double *herr = nullptr;   // w
    int64_t device_bytes = 0;
    std::vector<void *> allocations;
    rf_allocator alloc{};         // caller's device-memory callbacks (alloc == NULL: hipMalloc)
    std::string last_error;
    bool broken = false;
    bool shared_factors = false;  // F.tiles/perm/info belong to a batch's factor owner
    const rf_plan *adj_parent = nullptr;  // adjoint plan: the plan whose factors it transposes
    hipGraphExec_t fac_graph = nullptr;   // the factorization's launch sequence, recorded once
    // precision form: per-(shift, column) combine coefficients and per-(pole, column)
    // inner weights of the residual form
    zd *d_colcoef = nullptr;  // nq x w
    zd *d_colw = nullptr;     // p x w
    zd *d_lam = nullptr;      // w shifts of the residual
    bool colcoef_on = false;
};

// error helpers --------------------------------------------------------------
rf_status rf_fail(rf_plan *plan, rf_status s, const std::string &msg);

#define RF_HIP(plan, expr)                                                             \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            (plan)->broken = true;                                                     \
            return rf_fail((plan), RF_ERR_DEVICE, std::string(#expr) + ": " +          \
                                                      hipGetErrorString(_e));          \
        }                                                                              \
    } while (0)

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files); all enqueue on `s`
// ---------------------------------------------------------------------------
// band factorization / solves (rf_band.hip)
hipError_t launch_band_factor(const rf_plan &P, hipStream_t s);
// Z = sum_i w_i K_i^{-1} (B X): X n x ncols (ldx), Z n x ncols (ldz)
// apply_b = false: X already holds the right-hand sides (no B product); colw (device,
// [pole][ncols]) replaces w_i by a weight per pole and column.  The plan's precision
// selects the complex128 or complex64 factor tiles.
hipError_t launch_inner_apply(const rf_plan &P, const zd *X, int64_t ldx, int ncols,
                              zd *Z, int64_t ldz, hipStream_t s, bool apply_b = true,
                              const zd *colw = nullptr);
// launch_inner_apply with its work blocks in the library's file-scope device array
// instead of plan buffers (no allocation); columns go in chunks that fit the array.
// hipErrorInvalidValue if a single column does not fit.
hipError_t launch_inner_apply_static(const rf_plan &P, const zd *X, int64_t ldx, int ncols,
                                     zd *Z, int64_t ldz, hipStream_t s);
size_t inner_scratch_capacity();                    // bytes of that array
size_t inner_scratch_per_column(const rf_plan &P);  // its bytes per column, unaligned
// the adjoint plan P's tiles and row orders from the factorization of `parent`
// (P's pole i is the conjugate of parent's pole p-1-i): conjugate-transposed tiles
hipError_t launch_tiles_adjoint(const rf_plan &P, const rf_plan &parent, hipStream_t s);
// cluster solve over fused tiles (rf_cluster.hip)
struct ClusterSolve {
    const zd *X; int64_t ldx;      // right-hand sides before B, or B X itself (bdiag null)
    const zd *bdiag;               // diagonal of B, or null (then X holds B X)
    zd *stage;                     // npad x ncols: B X when bdiag is set
    int64_t x_pole_stride;         // 0: one block for all poles
    const zd *colw;                // or null: [pole][ncols] weights
    zd *zbuf, *xpart;              // [pole][npad x ncols] each
    int ncols;
    int unit_weight, accumulate;
};
bool cluster_solve_supported(int nb);              // tile sizes 64, 128, 256
int cluster_slots_max(int nb, int num_cu);         // clusters in flight at most
size_t cluster_xchg_elems(int nb, int num_cu);     // complex entries of the exchange area
size_t cluster_flag_words(int nb, int num_cu);     // 64-bit sequence flags
hipError_t cluster_gate_init(int device);          // once per device, before any launch
// F.ftiles from F.tiles (complex128 factors of every pole): M, W, V1, V2
hipError_t launch_fused_tiles(const rf_plan &P, hipStream_t s);
// xpart_i = w_i K_i^{-1} (B X) for every pole (or the unit-weight / accumulating forms)
hipError_t launch_cluster_solve(const rf_plan &P, const ClusterSolve &cs, hipStream_t s);
// complex64 copy of the factor tiles (after the complex128 factorization)
hipError_t launch_tiles_to_c64(const rf_plan &P, hipStream_t s);

// dense kernels (rf_dense.hip)
// Batched operands: entry t of operand X is at X + (flags & kMapX ? map[t] : t) * sX.
constexpr int kMapA = 1, kMapB = 2, kMapC = 4;
// C (m x k, ldc) = alpha * A^H B + beta * C, A: n x m (lda), B: n x k (ldb); batched by `batch`
// with strides; reduction over n uses split-N partials in `work`.
hipError_t launch_gemm_cn(int64_t n, int m, int k, zd alpha, const zd *A, int64_t lda,
                          int64_t sA, const zd *B, int64_t ldb, int64_t sB, zd beta, zd *C,
                          int64_t ldc, int64_t sC, int batch, zd *work, int64_t work_elems,
                          hipStream_t s, const int *map = nullptr, int flags = 0);
// C (n x k) = alpha * A (n x m) * B (m x k) + beta * C; batched
hipError_t launch_gemm_nn(int64_t n, int m, int k, zd alpha, const zd *A, int64_t lda,
                          int64_t sA, const zd *B, int64_t ldb, int64_t sB, zd beta, zd *C,
                          int64_t ldc, int64_t sC, int batch, hipStream_t s,
                          const int *map = nullptr, int flags = 0);
// Cholesky S = R^H R of batch Hermitian k x k matrices (ld k): R to Rout, R^{-1} to Rinv;
// status[t] != 0 on breakdown, dratio[t] = min R_ii / max R_ii.  For k <= 64 the
// factorization runs in LDS and S is left intact (map: A -> S, B -> Rout, C -> Rinv);
// for k > 64 S is overwritten and no map is allowed.
hipError_t launch_chol_inv(int k, zd *S, int64_t sS, zd *Rout, int64_t sR, zd *Rinv,
                           int64_t sRi, int batch, int *status, double *dratio,
                           double shift_rel, hipStream_t s, const int *map = nullptr,
                           int flags = 0);
// C (m x k) += alpha * A (m x k); batched (map: A, C)
hipError_t launch_add_block(int m, int k, zd alpha, const zd *A, int64_t lda, int64_t sA, zd *C,
                            int64_t ldc, int64_t sC, int batch, hipStream_t s,
                            const int *map = nullptr, int flags = 0);
// dst (n x ncols) = src; batched (map: A -> src, C -> dst)
hipError_t launch_copy_block(int64_t n, int ncols, const zd *src, int64_t lds, int64_t sS,
                             zd *dst, int64_t ldd, int64_t sD, int batch, hipStream_t s,
                             const int *map = nullptr, int flags = 0);
hipError_t launch_copy_cols(int64_t n, int ncols, const zd *src, int64_t lds, zd *dst,
                            int64_t ldd, hipStream_t s);
// d[i] = sum_r conj(Y[r, pair[i]]) * BX[r, i], i < s   (one workgroup per i)
hipError_t launch_paired_dots(int64_t n, int s, const zd *Y, int64_t ldy, const int *pair,
                              const zd *BX, int64_t ldb, zd *d, hipStream_t st);
// out[e] = sum_i coef[i] * conj(Y[row(e), pair[i]]) * X[col(e), i] over the stored entries e
// of M (CSR order)
hipError_t launch_sampled_outer(const DevCsr &M, int s, const zd *coef, const zd *Y, int64_t ldy,
                                const int *pair, const zd *X, int64_t ldx, zd *out,
                                hipStream_t st);
hipError_t launch_spmm(const DevCsr &M, int ncols, const zd *X, int64_t ldx, zd *Y,
                       int64_t ldy, hipStream_t s);
// Z[:, c] = X[:, c] - lam[c] Y[:, c]
hipError_t launch_sub_diag(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *Y,
                           int64_t ldy, const zd *lam, zd *Z, int64_t ldz, hipStream_t s);
// Z[:, c] += alpha[c] X[:, c]
hipError_t launch_add_diag(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *alpha, zd *Z,
                           int64_t ldz, hipStream_t s);
// Y = A X - sigma * B X   (all n x ncols)
hipError_t launch_axpby_cols(int64_t n, int ncols, zd alpha, const zd *X, int64_t ldx,
                             zd beta, const zd *Y, int64_t ldy, zd *Z, int64_t ldz,
                             hipStream_t s);
// column 2-norms of (X - Y diag(lam)) (Y may be null) -> out[c]
hipError_t launch_colnorms(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *Y,
                           int64_t ldy, const zd *lam, double *out, hipStream_t s);
hipError_t launch_inv_pos(int m, const double *src, double *dst, double other, hipStream_t s);
hipError_t launch_scale_cols(int64_t n, int ncols, zd *X, int64_t ldx, const double *inv,
                             hipStream_t s);
hipError_t launch_gaussian(int64_t n, int ncols, zd *X, int64_t ldx, uint64_t seed,
                           hipStream_t s);
// block-GMRES least-squares update for step j (see rf_dense.hip)
hipError_t launch_ls_update(const rf_plan &P, int j, const int *active, int nact,
                            hipStream_t s);
hipError_t launch_ls_solve(const rf_plan &P, int m, const int *active, int nact,
                           hipStream_t s);

// host QZ (rf_qz.cpp): eigenvalues and right eigenvectors of the pencil (A, B),
// both n x n column-major complex; vr gets eigenvectors (columns, unit 2-norm).
#include "rf_qz.h"
