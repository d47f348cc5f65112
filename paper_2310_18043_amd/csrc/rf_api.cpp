// C ABI of rfeig: plan creation, factorization, the composite filter and the
// subspace iteration (Chen & Li, Alg. composite, Sec. 3.2).  Host code; every
// step on the n-sized data runs in the kernels of rf_band.hip and rf_dense.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "rf_common.h"

namespace {

const double kPi = 3.14159265358979323846;

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

template <typename T>
rf_status dalloc(rf_plan *P, T **ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) return RF_OK;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return rf_fail(P, RF_ERR_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                            " bytes failed: " + hipGetErrorString(e));
    }
    P->allocations.push_back(p);
    P->device_bytes += int64_t(count * sizeof(T));
    *ptr = static_cast<T *>(p);
    return RF_OK;
}

#define RF_TRY(expr)                          \
    do {                                      \
        rf_status _s = (expr);                \
        if (_s != RF_OK) return _s;           \
    } while (0)

zd Z(double re, double im = 0.0) { return zmake(re, im); }

bool csr_ok(const rf_csr *M) {
    if (!M || M->n <= 0 || M->nnz < 0 || !M->rowptr) return false;
    if (M->nnz > 0 && (!M->colind || !M->val)) return false;
    if (M->rowptr[0] != 0 || M->rowptr[M->n] != M->nnz) return false;
    for (int32_t i = 0; i < M->n; ++i)
        if (M->rowptr[i + 1] < M->rowptr[i]) return false;
    for (int64_t e = 0; e < M->nnz; ++e) {
        if (M->colind[e] < 0 || M->colind[e] >= M->n) return false;
        if (!std::isfinite(M->val[2 * e]) || !std::isfinite(M->val[2 * e + 1])) return false;
    }
    return true;
}

void band_extent(const rf_csr *M, int &kl, int &ku) {
    for (int32_t i = 0; i < M->n; ++i)
        for (int64_t e = M->rowptr[i]; e < M->rowptr[i + 1]; ++e) {
            int d = i - M->colind[e];
            kl = std::max(kl, d);
            ku = std::max(ku, -d);
        }
}

rf_status upload_csr(rf_plan *P, const rf_csr *M, DevCsr &D) {
    D.n = M->n;
    D.nnz = M->nnz;
    RF_TRY(dalloc(P, &D.rowptr, size_t(M->n) + 1));
    RF_TRY(dalloc(P, &D.colind, size_t(std::max<int64_t>(M->nnz, 1))));
    RF_TRY(dalloc(P, &D.val, size_t(std::max<int64_t>(M->nnz, 1))));
    RF_HIP(P, hipMemcpy(D.rowptr, M->rowptr, sizeof(int32_t) * (M->n + 1), hipMemcpyHostToDevice));
    if (M->nnz > 0) {
        RF_HIP(P, hipMemcpy(D.colind, M->colind, sizeof(int32_t) * M->nnz, hipMemcpyHostToDevice));
        RF_HIP(P, hipMemcpy(D.val, M->val, sizeof(zd) * M->nnz, hipMemcpyHostToDevice));
    }
    // diagonal fast path: exactly one stored entry per row, on the diagonal
    bool diag = (M->nnz == M->n);
    for (int32_t i = 0; diag && i < M->n; ++i)
        diag = (M->rowptr[i + 1] - M->rowptr[i] == 1) && (M->colind[M->rowptr[i]] == i);
    D.diagonal = diag;
    if (diag) D.dval = D.val;
    return RF_OK;
}

}  // namespace

rf_status rf_fail(rf_plan *plan, rf_status s, const std::string &msg) {
    if (plan) plan->last_error = msg;
    return s;
}

extern "C" {

void rf_default_opts(rf_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->c_re = 0.0; o->c_im = 0.0; o->r = 1.0;
    o->p = 4; o->q = 8; o->w = 32;
    o->sigma_re = std::numeric_limits<double>::quiet_NaN();
    o->sigma_im = 0.0;
    o->tau = 1e-10; o->tau_g = 1e-2; o->gmres_tol = 1e-12;
    o->max_subspace_it = 10;
    o->max_krylov_blocks = 150;
    o->subblock = 0;
    o->expected_count = -1;
    o->tile = 0;
    o->trsm_cols = 0;
    o->seed = 0;
}

const char *rf_status_str(rf_status s) {
    switch (s) {
        case RF_OK: return "ok";
        case RF_ERR_ARG: return "invalid argument";
        case RF_ERR_NOMEM: return "device out of memory";
        case RF_ERR_SINGULAR: return "exactly singular shifted pencil (pole on an eigenvalue)";
        case RF_ERR_NOCONV: return "iteration cap reached before convergence";
        case RF_ERR_DEVICE: return "device error";
        case RF_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

const char *rf_last_error(rf_plan_t plan) { return plan ? plan->last_error.c_str() : ""; }

int64_t rf_plan_n(rf_plan_t plan) { return plan ? plan->n : -1; }

int64_t rf_plan_device_bytes(rf_plan_t plan) { return plan ? plan->device_bytes : -1; }

void rf_plan_destroy(rf_plan_t plan) {
    if (!plan) return;
    if (!plan->broken) (void)hipStreamSynchronize(plan->stream);
    for (void *p : plan->allocations) (void)hipFree(p);
    delete plan;
}

rf_status rf_plan_create(const rf_csr *A, const rf_csr *B, const rf_opts *opts,
                         void *hip_stream, rf_plan_t *out) {
    if (!out) return RF_ERR_ARG;
    *out = nullptr;
    if (!opts || !csr_ok(A) || !csr_ok(B) || A->n != B->n) return RF_ERR_ARG;
    const rf_opts &o = *opts;
    if (!(o.r > 0.0) || !std::isfinite(o.c_re) || !std::isfinite(o.c_im) || !std::isfinite(o.r))
        return RF_ERR_ARG;
    if (o.p < 1 || o.q < 1 || o.w < 1 || o.w > A->n) return RF_ERR_ARG;
    if (!(o.gmres_tol > 0.0) || !(o.tau > 0.0) || !(o.tau_g > 0.0)) return RF_ERR_ARG;
    if (o.max_krylov_blocks < 1 || o.max_subspace_it < 1) return RF_ERR_ARG;
    if (o.subblock < 0 || (o.subblock > 0 && (o.w % o.subblock != 0 || o.subblock > 32 ||
                                              (256 % o.subblock) != 0)))
        return RF_ERR_ARG;
    if (o.tile < 0 || o.tile > 256 || (o.tile > 0 && o.tile % 16 != 0)) return RF_ERR_ARG;
    if (o.trsm_cols < 0 || o.trsm_cols > 8) return RF_ERR_ARG;

    rf_plan *P = new rf_plan();
    P->opts = o;
    P->n = A->n;
    P->stream = static_cast<hipStream_t>(hip_stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        delete P;
        return RF_ERR_DEVICE;
    }
    P->device = dev;
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            P->max_lds = lds;
        else
            (void)hipGetLastError();
    }
    auto fail = [&](rf_status s) {
        *out = P;  // keep the plan so the caller can read rf_last_error, then destroy
        return s;
    };

    // band extents of pattern(A) U pattern(B) and the tile size
    int kl = 0, ku = 0;
    band_extent(A, kl, ku);
    band_extent(B, kl, ku);
    P->kl = kl; P->ku = ku;
    int nb = o.tile;
    if (nb == 0) nb = std::max(16, ((std::max(std::max(kl, ku), 1) + 15) / 16) * 16);
    if (nb < std::max(kl, ku)) {
        rf_fail(P, RF_ERR_ARG, "tile smaller than the bandwidth");
        return fail(RF_ERR_ARG);
    }
    if (nb > 256) {
        rf_fail(P, RF_ERR_ARG, "bandwidth above 256 is not supported by the band kernels");
        return fail(RF_ERR_ARG);
    }
    P->F.nb = nb;
    P->F.nblk = int((P->n + nb - 1) / nb);
    P->F.tile_elems = int64_t(nb) * nb;
    const int64_t npad = int64_t(P->F.nblk) * nb;

    // inner rule: eq. pwtp, theta_i = (2i-1) pi / p
    const std::complex<double> c(o.c_re, o.c_im);
    for (int i = 1; i <= o.p; ++i) {
        double th = (2.0 * i - 1.0) * kPi / o.p;
        std::complex<double> e = std::polar(1.0, th);
        std::complex<double> pole = c + o.r * e, wgt = o.r * e / double(o.p);
        P->poles.push_back(Z(pole.real(), pole.imag()));
        P->weights.push_back(Z(wgt.real(), wgt.imag()));
    }
    // outer rule: sigma_j roots of z^q = -1; s_j = 1/(1+sigma_j),
    // c'_j = (1/q) sigma_j/(1+sigma_j); the root -1 (odd q) contributes (1/q) G.
    for (int j = 1; j <= o.q; ++j) {
        std::complex<double> sg = std::polar(1.0, (2.0 * j - 1.0) * kPi / o.q);
        if (std::abs(1.0 + sg) < 1e-12) { P->oextra = 1.0 / o.q; continue; }
        std::complex<double> sj = 1.0 / (1.0 + sg), cj = sg / (double(o.q) * (1.0 + sg));
        P->shifts.push_back(Z(sj.real(), sj.imag()));
        P->oweights.push_back(Z(cj.real(), cj.imag()));
    }
    const int nq = int(P->shifts.size());

    // Krylov sub-block width
    int b = o.subblock;
    if (b == 0) {
        b = 32;
        while (b > 1 && o.w % b != 0) b /= 2;
        if (o.w < b) b = o.w;
        while (b > 1 && (o.w % b != 0 || 256 % b != 0)) --b;
    }
    P->b = b;
    P->nsub = o.w / b;
    P->mmax = o.max_krylov_blocks;

    rf_status st;
#define ALLOC(ptr, cnt) do { st = dalloc(P, &(ptr), size_t(cnt)); if (st != RF_OK) return fail(st); } while (0)
    st = upload_csr(P, A, P->A); if (st != RF_OK) return fail(st);
    st = upload_csr(P, B, P->B); if (st != RF_OK) return fail(st);
    ALLOC(P->d_poles, o.p);
    ALLOC(P->d_weights, o.p);
    ALLOC(P->d_shifts, std::max(nq, 1));
    ALLOC(P->d_oweights, std::max(nq, 1));
    if (hipMemcpy(P->d_poles, P->poles.data(), sizeof(zd) * o.p, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->d_weights, P->weights.data(), sizeof(zd) * o.p, hipMemcpyHostToDevice) != hipSuccess ||
        (nq > 0 && hipMemcpy(P->d_shifts, P->shifts.data(), sizeof(zd) * nq, hipMemcpyHostToDevice) != hipSuccess) ||
        (nq > 0 && hipMemcpy(P->d_oweights, P->oweights.data(), sizeof(zd) * nq, hipMemcpyHostToDevice) != hipSuccess)) {
        P->broken = true;
        rf_fail(P, RF_ERR_DEVICE, "copy of the rule coefficients failed");
        return fail(RF_ERR_DEVICE);
    }
    const int64_t te = P->F.tile_elems;
    ALLOC(P->F.tiles, int64_t(o.p) * P->F.nblk * 5 * te);
    ALLOC(P->F.perm, int64_t(o.p) * P->F.nblk * 2 * nb);
    ALLOC(P->F.window, int64_t(o.p) * (2 * nb) * (3 * nb));
    ALLOC(P->F.info, o.p);
    const int64_t n = P->n, w = o.w;
    ALLOC(P->rhs, npad * w);
    ALLOC(P->ypart, int64_t(o.p) * npad * w);
    ALLOC(P->xpart, int64_t(o.p) * npad * w);
    ALLOC(P->ytil, n * w);
    ALLOC(P->tmp, n * w);
    ALLOC(P->Wk, n * w);
    ALLOC(P->Gin, n * w);
    const int64_t mb = int64_t(P->mmax) * b, ldc = int64_t(P->mmax + 1) * b;
    ALLOC(P->V, int64_t(P->nsub) * n * ldc);
    ALLOC(P->Hm, int64_t(P->nsub) * ldc * mb);
    ALLOC(P->R0, int64_t(P->nsub) * b * b);
    const int64_t nqs = int64_t(std::max(nq, 1)) * P->nsub;
    ALLOC(P->lsQ, nqs * P->mmax * 4 * b * b);
    ALLOC(P->lsR, nqs * mb * mb);
    ALLOC(P->lsG, nqs * ldc * b);
    ALLOC(P->lsWork, nqs * ldc * b);
    ALLOC(P->lsY, nqs * mb * b);
    ALLOC(P->ycomb, int64_t(P->nsub) * mb * b);
    ALLOC(P->resid, nqs * b);
    ALLOC(P->r0norm, int64_t(P->nsub) * b);
    ALLOC(P->colnorm, std::max<int64_t>(w, 1) * 2);
    ALLOC(P->small, 8 * w * w + 8 * b * b);
    ALLOC(P->hbuf, ldc * b);
    ALLOC(P->rnew, int64_t(b) * b);
    ALLOC(P->ident, int64_t(b) * b);
    {
        std::vector<zd> I(size_t(b) * b, Z(0));
        for (int i = 0; i < b; ++i) I[i + size_t(i) * b] = Z(1);
        if (hipMemcpy(P->ident, I.data(), sizeof(zd) * I.size(), hipMemcpyHostToDevice) != hipSuccess) {
            P->broken = true;
            rf_fail(P, RF_ERR_DEVICE, "copy of the identity block failed");
            return fail(RF_ERR_DEVICE);
        }
    }
    P->partial_elems = std::max<int64_t>(int64_t(1) << 22, 16 * w * w);
    ALLOC(P->partial, P->partial_elems);
    ALLOC(P->flag, 64 + w);
    ALLOC(P->hV, n * w);
    ALLOC(P->hAV, n * w);
    ALLOC(P->hBV, n * w);
    ALLOC(P->hW, n * w);
    ALLOC(P->hX, n * w);
    ALLOC(P->hproj, 2 * w * w);
    ALLOC(P->herr, 2 * w);
#undef ALLOC
    *out = P;
    return RF_OK;
}

rf_status rf_factor_shifts(rf_plan_t P) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    RF_HIP(P, launch_band_factor(*P, P->stream));
    std::vector<int32_t> info(P->opts.p);
    RF_HIP(P, hipMemcpyAsync(info.data(), P->F.info, sizeof(int32_t) * P->opts.p,
                             hipMemcpyDeviceToHost, P->stream));
    RF_HIP(P, hipStreamSynchronize(P->stream));
    for (int i = 0; i < P->opts.p; ++i)
        if (info[i] != 0) {
            P->F.ready = false;
            return rf_fail(P, RF_ERR_SINGULAR,
                           "zero pivot in the factorization of pole " + std::to_string(i) +
                               " at column " + std::to_string(info[i] - 1));
        }
    P->F.ready = true;
    return RF_OK;
}

rf_status rf_apply_inner(rf_plan_t P, const void *X, int64_t ldx, int32_t ncols, void *Zp,
                         int64_t ldz) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!P->F.ready) return rf_fail(P, RF_ERR_STATE, "rf_factor_shifts has not succeeded");
    if (!X || !Zp || ncols < 0 || ncols > P->opts.w || ldx < P->n || ldz < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad block arguments");
    if (ncols == 0) return RF_OK;
    RF_HIP(P, launch_inner_apply(*P, static_cast<const zd *>(X), ldx, ncols, static_cast<zd *>(Zp),
                                 ldz, P->stream));
    RF_HIP(P, hipStreamSynchronize(P->stream));
    return RF_OK;
}

namespace {

// Orthonormalise the n x k block Wb (ld n) in place by CholeskyQR2 (shifted
// CholeskyQR3 if the Gram matrix is numerically indefinite).  Rout (k x k, on the
// device) receives the triangular factor with Wb_in = Q Rout.  tmp: n x k scratch.
rf_status cholqr(rf_plan *P, zd *Wb, int64_t n, int k, zd *Rout, zd *tmp) {
    hipStream_t s = P->stream;
    zd *S = P->small;                      // k x k
    zd *R1 = S + int64_t(k) * k;
    zd *R1i = R1 + int64_t(k) * k;
    zd *R2 = R1i + int64_t(k) * k;
    zd *R2i = R2 + int64_t(k) * k;
    zd *Racc = R2i + int64_t(k) * k;
    int *status = P->flag;
    const int kk = k;
    // first pass (retried with a shift on breakdown)
    for (int attempt = 0; attempt < 2; ++attempt) {
        double shift = attempt == 0 ? 0.0 : 11.0 * (double(n) * kk + double(kk) * (kk + 1)) * 1.1102230246251565e-16;
        RF_HIP(P, launch_gemm_cn(n, kk, kk, Z(1), Wb, n, 0, Wb, n, 0, Z(0), S, kk, 0, 1, P->partial,
                                 P->partial_elems, s));
        RF_HIP(P, launch_chol_inv(kk, S, 0, R1, 0, R1i, 0, 1, status, shift, s));
        int hstat = 0;
        RF_HIP(P, hipMemcpyAsync(&hstat, status, sizeof(int), hipMemcpyDeviceToHost, s));
        RF_HIP(P, hipStreamSynchronize(s));
        if (hstat == 0) break;
        if (attempt == 1) return rf_fail(P, RF_ERR_NOCONV, "CholeskyQR breakdown (rank-deficient block)");
    }
    RF_HIP(P, launch_gemm_nn(n, kk, kk, Z(1), Wb, n, 0, R1i, kk, 0, Z(0), tmp, n, 0, 1, s));
    // two more passes on the (now well-conditioned) block
    RF_HIP(P, hipMemcpyAsync(Racc, R1, sizeof(zd) * kk * kk, hipMemcpyDeviceToDevice, s));
    zd *src = tmp, *dst = Wb;
    for (int pass = 0; pass < 2; ++pass) {
        RF_HIP(P, launch_gemm_cn(n, kk, kk, Z(1), src, n, 0, src, n, 0, Z(0), S, kk, 0, 1, P->partial,
                                 P->partial_elems, s));
        RF_HIP(P, launch_chol_inv(kk, S, 0, R2, 0, R2i, 0, 1, status, 0.0, s));
        RF_HIP(P, launch_gemm_nn(n, kk, kk, Z(1), src, n, 0, R2i, kk, 0, Z(0), dst, n, 0, 1, s));
        // Racc <- R2 * Racc (via R1 scratch)
        RF_HIP(P, launch_gemm_nn(kk, kk, kk, Z(1), R2, kk, 0, Racc, kk, 0, Z(0), R1, kk, 0, 1, s));
        RF_HIP(P, hipMemcpyAsync(Racc, R1, sizeof(zd) * kk * kk, hipMemcpyDeviceToDevice, s));
        std::swap(src, dst);
    }
    // after two passes the result is back in Wb (src after the final swap is Wb)
    if (src != Wb) RF_HIP(P, hipMemcpyAsync(Wb, src, sizeof(zd) * n * kk, hipMemcpyDeviceToDevice, s));
    if (Rout) RF_HIP(P, hipMemcpyAsync(Rout, Racc, sizeof(zd) * kk * kk, hipMemcpyDeviceToDevice, s));
    int hstat = 0;
    RF_HIP(P, hipMemcpyAsync(&hstat, status, sizeof(int), hipMemcpyDeviceToHost, s));
    RF_HIP(P, hipStreamSynchronize(s));
    if (hstat != 0) return rf_fail(P, RF_ERR_NOCONV, "CholeskyQR breakdown in the second pass");
    return RF_OK;
}

// U = sum_j c'_j (G - s_j I)^{-1} G(Y) by block multi-shift GMRES.
rf_status filter_core(rf_plan *P, const zd *Y, int64_t ldy, zd *U, int64_t ldu,
                      rf_filter_info *info) {
    const double t0 = now_ms();
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w, b = P->b, nsub = P->nsub, mmax = P->mmax;
    const int nq = int(P->shifts.size());
    const int64_t ldc = int64_t(mmax + 1) * b, mbmax = int64_t(mmax) * b;
    const int64_t vstride = n * ldc;                 // per sub-block basis
    const int64_t hstride = ldc * mbmax;
    (void)w;
    int64_t inner_cols = 0;

    // Ytilde = G(Y)
    RF_HIP(P, launch_inner_apply(*P, Y, ldy, w, P->ytil, n, s));
    inner_cols += w;
    // column norms of Ytilde (per sub-block) for relative residuals
    RF_HIP(P, launch_colnorms(n, w, P->ytil, n, nullptr, 0, nullptr, P->r0norm, s));
    // V_sb[0] R0_sb = Ytilde_sb
    for (int sb = 0; sb < nsub; ++sb) {
        zd *V0 = P->V + sb * vstride;
        RF_HIP(P, launch_copy_cols(n, b, P->ytil + int64_t(sb) * b * n, n, V0, n, s));
        RF_TRY(cholqr(P, V0, n, b, P->R0 + int64_t(sb) * b * b, P->tmp));
    }
    // right-hand sides E1 R0 per (shift, sub-block); Hessenberg columns are
    // cleared step by step
    if (nq > 0) {
        RF_HIP(P, hipMemsetAsync(P->lsG, 0, sizeof(zd) * int64_t(nq) * nsub * ldc * b, s));
        for (int l = 0; l < nq; ++l)
            for (int sb = 0; sb < nsub; ++sb)
                RF_HIP(P, hipMemcpy2DAsync(P->lsG + (int64_t(l) * nsub + sb) * ldc * b, ldc * sizeof(zd),
                                           P->R0 + int64_t(sb) * b * b, b * sizeof(zd), b * sizeof(zd), b,
                                           hipMemcpyDeviceToDevice, s));
    }
    std::vector<int> active(nsub), msteps(nsub, 0);
    std::iota(active.begin(), active.end(), 0);
    std::vector<double> resid(size_t(std::max(nq, 1)) * nsub * b);
    double worst_final = 0.0;
    bool all_conv = true;
    int steps = 0;
    int *d_active = P->flag + 16;
    if (nq == 0) active.clear();         // q = 1: the filter is (1/q) G(Y) only
    for (int j = 0; j < mmax && !active.empty(); ++j) {
        const int nact = int(active.size());
        // gather the newest basis block of every active sub-block
        for (int a = 0; a < nact; ++a) {
            int sb = active[a];
            RF_HIP(P, launch_copy_cols(n, b, P->V + sb * vstride + int64_t(j) * b * n, n,
                                       P->Gin + int64_t(a) * b * n, n, s));
        }
        RF_HIP(P, launch_inner_apply(*P, P->Gin, n, nact * b, P->Wk, n, s));
        inner_cols += int64_t(nact) * b;
        for (int a = 0; a < nact; ++a) {
            int sb = active[a];
            zd *Vs = P->V + sb * vstride;
            zd *Wb = P->Wk + int64_t(a) * b * n;
            zd *Hc = P->Hm + sb * hstride + int64_t(j) * b * ldc;     // block column j
            const int kb = (j + 1) * b;
            RF_HIP(P, hipMemset2DAsync(Hc, ldc * sizeof(zd), 0, (j + 2) * b * sizeof(zd), b, s));
            for (int pass = 0; pass < 2; ++pass) {   // block classical Gram-Schmidt, twice
                zd *h = P->hbuf;                                      // kb x b
                RF_HIP(P, launch_gemm_cn(n, kb, b, Z(1), Vs, n, 0, Wb, n, 0, Z(0), h, kb, 0, 1,
                                         P->partial, P->partial_elems, s));
                RF_HIP(P, launch_gemm_nn(n, kb, b, Z(-1), Vs, n, 0, h, kb, 0, Z(1), Wb, n, 0, 1, s));
                // H[0:kb, jb:(j+1)b] += h
                RF_HIP(P, launch_gemm_nn(kb, b, b, Z(1), h, kb, 0, P->ident, b, 0, Z(1), Hc, ldc, 0, 1, s));
            }
            // V_{j+1} R = W ;  H[(j+1)b:(j+2)b, jb:(j+1)b] = R
            zd *Rn = P->rnew;
            RF_TRY(cholqr(P, Wb, n, b, Rn, P->tmp));
            RF_HIP(P, launch_copy_cols(n, b, Wb, n, Vs + int64_t(j + 1) * b * n, n, s));
            RF_HIP(P, hipMemcpy2DAsync(Hc + int64_t(j + 1) * b, ldc * sizeof(zd), Rn, b * sizeof(zd),
                                       b * sizeof(zd), b, hipMemcpyDeviceToDevice, s));
        }
        // per-shift least squares update and residuals
        RF_HIP(P, hipMemcpyAsync(d_active, active.data(), sizeof(int) * nact, hipMemcpyHostToDevice, s));
        RF_HIP(P, launch_ls_update(*P, j, d_active, nact, s));
        RF_HIP(P, hipMemcpyAsync(resid.data(), P->resid, sizeof(double) * nq * nsub * b,
                                 hipMemcpyDeviceToHost, s));
        RF_HIP(P, hipStreamSynchronize(s));
        steps = j + 1;
        std::vector<int> still;
        for (int sb : active) {
            double worst = 0.0;
            for (int l = 0; l < nq; ++l)
                for (int c = 0; c < b; ++c) worst = std::max(worst, resid[(size_t(l) * nsub + sb) * b + c]);
            msteps[sb] = j + 1;
            if (!(worst <= P->opts.gmres_tol) && j + 1 < mmax) still.push_back(sb);
            else {
                if (!(worst <= P->opts.gmres_tol)) all_conv = false;
                worst_final = std::max(worst_final, worst);
            }
        }
        active.swap(still);
    }
    // solve the triangular systems, combine shifts, U_sb = V_sb Ycomb_sb
    for (int sb = 0; sb < nsub; ++sb) {
        const int m = msteps[sb];
        zd *Us = U + int64_t(sb) * b * ldu;
        if (m == 0) {
            RF_HIP(P, hipMemset2DAsync(Us, ldu * sizeof(zd), 0, n * sizeof(zd), b, s));
        } else {
            int one = sb;
            RF_HIP(P, hipMemcpyAsync(d_active, &one, sizeof(int), hipMemcpyHostToDevice, s));
            RF_HIP(P, launch_ls_solve(*P, m, d_active, 1, s));
            RF_HIP(P, launch_gemm_nn(n, m * b, b, Z(1), P->V + sb * vstride, n, 0,
                                     P->ycomb + int64_t(sb) * mbmax * b, mbmax, 0, Z(0), Us, ldu, 0, 1,
                                     s));
            RF_HIP(P, hipStreamSynchronize(s));
        }
        if (P->oextra != 0.0)
            RF_HIP(P, launch_axpby_cols(n, b, Z(1), Us, ldu, Z(P->oextra), P->ytil + int64_t(sb) * b * n,
                                        n, Us, ldu, s));
    }
    RF_HIP(P, hipStreamSynchronize(s));
    if (info) {
        info->krylov_steps = steps;
        info->converged = all_conv ? 1 : 0;
        info->max_residual = worst_final;
        info->inner_columns = inner_cols;
        info->ms_total = now_ms() - t0;
    }
    return all_conv ? RF_OK : RF_ERR_NOCONV;
}

}  // namespace

rf_status rf_filter_apply(rf_plan_t P, const void *Y, int64_t ldy, int32_t ncols, void *U,
                          int64_t ldu, rf_filter_info *info) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!P->F.ready) return rf_fail(P, RF_ERR_STATE, "rf_factor_shifts has not succeeded");
    if (!Y || !U || ncols != P->opts.w || ldy < P->n || ldu < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad block arguments (ncols must equal w)");
    return filter_core(P, static_cast<const zd *>(Y), ldy, static_cast<zd *>(U), ldu, info);
}

namespace {

// HSRR(A, B, U, sigma) (Sec. 2.1): Ritz values lam (host), unit-norm Ritz vectors in
// P->hX, errors e_i (eq. rel-error) in err (host).
rf_status hsrr(rf_plan *P, zd *U, std::vector<std::complex<double>> &lam,
               std::vector<double> &err) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w;
    const std::complex<double> sigma =
        std::isnan(P->opts.sigma_re) ? std::complex<double>(P->opts.c_re, P->opts.c_im)
                                     : std::complex<double>(P->opts.sigma_re, P->opts.sigma_im);
    // V = orth(U): normalise columns first (span unchanged), then CholeskyQR
    RF_HIP(P, launch_colnorms(n, w, U, n, nullptr, 0, nullptr, P->colnorm, s));
    std::vector<double> cn(w);
    RF_HIP(P, hipMemcpyAsync(cn.data(), P->colnorm, sizeof(double) * w, hipMemcpyDeviceToHost, s));
    RF_HIP(P, hipStreamSynchronize(s));
    for (auto &v : cn) v = v > 0.0 ? 1.0 / v : 1.0;
    RF_HIP(P, hipMemcpyAsync(P->colnorm, cn.data(), sizeof(double) * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_copy_cols(n, w, U, n, P->hV, n, s));
    RF_HIP(P, launch_scale_cols(n, w, P->hV, n, P->colnorm, s));
    RF_TRY(cholqr(P, P->hV, n, w, nullptr, P->tmp));
    // AV, BV, W = orth(AV - sigma BV)
    RF_HIP(P, launch_spmm(P->A, w, P->hV, n, P->hAV, n, s));
    RF_HIP(P, launch_spmm(P->B, w, P->hV, n, P->hBV, n, s));
    RF_HIP(P, launch_axpby_cols(n, w, Z(1), P->hAV, n, Z(-sigma.real(), -sigma.imag()), P->hBV, n,
                                P->hW, n, s));
    RF_TRY(cholqr(P, P->hW, n, w, nullptr, P->tmp));
    // projected pencil
    zd *Ah = P->hproj, *Bh = P->hproj + int64_t(w) * w;
    RF_HIP(P, launch_gemm_cn(n, w, w, Z(1), P->hW, n, 0, P->hAV, n, 0, Z(0), Ah, w, 0, 1, P->partial,
                             P->partial_elems, s));
    RF_HIP(P, launch_gemm_cn(n, w, w, Z(1), P->hW, n, 0, P->hBV, n, 0, Z(0), Bh, w, 0, 1, P->partial,
                             P->partial_elems, s));
    std::vector<zd> hA(size_t(w) * w), hB(size_t(w) * w), al(w), be(w), vr(size_t(w) * w);
    RF_HIP(P, hipMemcpyAsync(hA.data(), Ah, sizeof(zd) * w * w, hipMemcpyDeviceToHost, s));
    RF_HIP(P, hipMemcpyAsync(hB.data(), Bh, sizeof(zd) * w * w, hipMemcpyDeviceToHost, s));
    RF_HIP(P, hipStreamSynchronize(s));
    if (host_qz_eig(w, hA.data(), hB.data(), al.data(), be.data(), vr.data()) != 0)
        return rf_fail(P, RF_ERR_NOCONV, "QZ iteration did not converge");
    lam.resize(w);
    std::vector<zd> dlam(w);
    for (int i = 0; i < w; ++i) {
        std::complex<double> a(al[i].x, al[i].y), bb(be[i].x, be[i].y);
        lam[i] = (std::abs(bb) > 0.0) ? a / bb : std::complex<double>(INFINITY, 0.0);
        dlam[i] = Z(lam[i].real(), lam[i].imag());
    }
    // X = V (P_R V_R), unit columns
    zd *dvr = P->small;
    RF_HIP(P, hipMemcpyAsync(dvr, vr.data(), sizeof(zd) * w * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_gemm_nn(n, w, w, Z(1), P->hV, n, 0, dvr, w, 0, Z(0), P->hX, n, 0, 1, s));
    RF_HIP(P, launch_colnorms(n, w, P->hX, n, nullptr, 0, nullptr, P->colnorm, s));
    RF_HIP(P, hipMemcpyAsync(cn.data(), P->colnorm, sizeof(double) * w, hipMemcpyDeviceToHost, s));
    RF_HIP(P, hipStreamSynchronize(s));
    for (auto &v : cn) v = v > 0.0 ? 1.0 / v : 1.0;
    RF_HIP(P, hipMemcpyAsync(P->colnorm, cn.data(), sizeof(double) * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_scale_cols(n, w, P->hX, n, P->colnorm, s));
    // e_i = ||A x - lam B x|| / ((|c| + r) ||B x||)
    zd *dl = P->small + int64_t(w) * w;
    RF_HIP(P, hipMemcpyAsync(dl, dlam.data(), sizeof(zd) * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_spmm(P->A, w, P->hX, n, P->hAV, n, s));
    RF_HIP(P, launch_spmm(P->B, w, P->hX, n, P->hBV, n, s));
    RF_HIP(P, launch_colnorms(n, w, P->hAV, n, P->hBV, n, dl, P->herr, s));
    RF_HIP(P, launch_colnorms(n, w, P->hBV, n, nullptr, 0, nullptr, P->herr + w, s));
    std::vector<double> e2(2 * w);
    RF_HIP(P, hipMemcpyAsync(e2.data(), P->herr, sizeof(double) * 2 * w, hipMemcpyDeviceToHost, s));
    RF_HIP(P, hipStreamSynchronize(s));
    const double scale = std::abs(std::complex<double>(P->opts.c_re, P->opts.c_im)) + P->opts.r;
    err.resize(w);
    for (int i = 0; i < w; ++i) {
        double den = scale * e2[w + i];
        err[i] = (den > 0.0 && std::isfinite(lam[i].real())) ? e2[i] / den : INFINITY;
    }
    return RF_OK;
}

}  // namespace

rf_status rf_solve_region(rf_plan_t P, const void *Y0, int64_t ldy, rf_result *res) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!res || !res->lambda || !res->X || !res->err || !res->flags || res->ldx < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad result buffers");
    if (Y0 && ldy < P->n) return rf_fail(P, RF_ERR_ARG, "bad start block");
    const double t_start = now_ms();
    if (!P->F.ready) RF_TRY(rf_factor_shifts(P));
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w;
    zd *Y = P->hX;   // current block (Ritz vectors after the first sweep)
    if (Y0) RF_HIP(P, launch_copy_cols(n, w, static_cast<const zd *>(Y0), ldy, Y, n, s));
    else RF_HIP(P, launch_gaussian(n, w, Y, n, P->opts.seed, s));
    // Y = orth(Y)  (Alg. composite: orthonormal random start)
    RF_TRY(cholqr(P, Y, n, w, nullptr, P->tmp));
    const std::complex<double> c(P->opts.c_re, P->opts.c_im);
    const double r = P->opts.r;
    std::vector<std::complex<double>> lam;
    std::vector<double> err;
    int prev = -1, t = 0;
    bool converged = false;
    double ms_filter = 0.0, ms_hsrr = 0.0;
    std::vector<int> flags(w);
    for (t = 1; t <= P->opts.max_subspace_it; ++t) {
        rf_filter_info fi;
        double t1 = now_ms();
        // U lands in P->Wk? no: Wk is Krylov scratch; use hW as the output block
        rf_status fs = filter_core(P, Y, n, P->hW, n, &fi);
        if (fs != RF_OK && fs != RF_ERR_NOCONV) return fs;
        // copy U out of hW before HSRR reuses it
        RF_HIP(P, launch_copy_cols(n, w, P->hW, n, P->ytil, n, s));
        double t2 = now_ms();
        ms_filter += t2 - t1;
        if (t <= 16) res->krylov_steps[t - 1] = fi.krylov_steps;
        RF_TRY(hsrr(P, P->ytil, lam, err));
        ms_hsrr += now_ms() - t2;
        int count = 0;
        bool all_small = true;
        for (int i = 0; i < w; ++i) {
            bool inside = std::abs(lam[i] - c) < r;
            bool filt = inside && err[i] < P->opts.tau_g;
            flags[i] = (inside ? 1 : 0) | (filt ? 2 : 0) | (err[i] <= P->opts.tau ? 4 : 0);
            if (filt) { ++count; if (!(err[i] <= P->opts.tau)) all_small = false; }
        }
        if (all_small && (count == prev || (t == 1 && P->opts.expected_count >= 0 &&
                                            count == P->opts.expected_count))) {
            converged = true;
            break;
        }
        prev = count;
    }
    if (t > P->opts.max_subspace_it) t = P->opts.max_subspace_it;
    // order: converged pairs inside D first, then the rest
    std::vector<int> order(w);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b2) {
        bool ga = (flags[a] & 7) == 7, gb = (flags[b2] & 7) == 7;
        return ga > gb;
    });
    int count = 0;
    for (int i = 0; i < w; ++i) {
        int k = order[i];
        res->lambda[2 * i] = lam[k].real();
        res->lambda[2 * i + 1] = lam[k].imag();
        res->err[i] = err[k];
        res->flags[i] = flags[k];
        if ((flags[k] & 7) == 7) ++count;
        RF_HIP(P, hipMemcpyAsync(static_cast<zd *>(res->X) + int64_t(i) * res->ldx, P->hX + int64_t(k) * n,
                                 sizeof(zd) * n, hipMemcpyDeviceToDevice, s));
    }
    RF_HIP(P, hipStreamSynchronize(s));
    res->count = count;
    res->sweeps = t;
    res->converged = converged ? 1 : 0;
    res->ms_filter = ms_filter;
    res->ms_hsrr = ms_hsrr;
    (void)t_start;
    return converged ? RF_OK : RF_ERR_NOCONV;
}

}  // extern "C"
