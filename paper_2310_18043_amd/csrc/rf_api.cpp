// C ABI of rfeig: plan creation, factorization, the composite filter and the
// subspace iteration (Chen & Li, Alg. composite, Sec. 3.2).  Host code; every
// step on the n-sized data runs in the kernels of rf_band.hip and rf_dense.hip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <tuple>
#include <limits>
#include <numeric>
#include <string>
#include <thread>
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
    const size_t bytes = count * sizeof(T);
    if (P->alloc.alloc) {
        p = P->alloc.alloc(bytes, P->alloc.ctx);
        if (!p)
            return rf_fail(P, RF_ERR_NOMEM, "the caller's allocator returned no memory for " +
                                                std::to_string(bytes) + " bytes");
        if (reinterpret_cast<uintptr_t>(p) % 16 != 0) {
            P->alloc.free(p, P->alloc.ctx);
            return rf_fail(P, RF_ERR_NOMEM, "the caller's allocator returned memory aligned to "
                                            "less than 16 bytes");
        }
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return rf_fail(P, RF_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) +
                                                " bytes failed: " + hipGetErrorString(e));
        }
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

// Outer trapezoidal rule with q nodes (Thm. Rcrm, sign as in its proof): sigma_j the
// roots of z^q = -1, shifts s_j = 1/(1+sigma_j), weights c'_j = sigma_j/(q(1+sigma_j));
// the root -1 (odd q) contributes the term (1/q) G instead of a shift.
void outer_rule(int q, std::vector<zd> &shifts, std::vector<zd> &weights, double &extra) {
    shifts.clear();
    weights.clear();
    extra = 0.0;
    for (int j = 1; j <= q; ++j) {
        std::complex<double> sg = std::polar(1.0, (2.0 * j - 1.0) * kPi / q);
        if (std::abs(1.0 + sg) < 1e-12) { extra = 1.0 / q; continue; }
        std::complex<double> sj = 1.0 / (1.0 + sg), cj = sg / (double(q) * (1.0 + sg));
        shifts.push_back(Z(sj.real(), sj.imag()));
        weights.push_back(Z(cj.real(), cj.imag()));
    }
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
    // copies on the plan's stream, never the legacy stream: a legacy-stream operation would
    // depend on every blocking stream, and so fail while another thread records a graph
    // on one of its own
    RF_HIP(P, hipMemcpyAsync(D.rowptr, M->rowptr, sizeof(int32_t) * (M->n + 1),
                             hipMemcpyHostToDevice, P->stream));
    if (M->nnz > 0) {
        RF_HIP(P, hipMemcpyAsync(D.colind, M->colind, sizeof(int32_t) * M->nnz,
                                 hipMemcpyHostToDevice, P->stream));
        RF_HIP(P, hipMemcpyAsync(D.val, M->val, sizeof(zd) * M->nnz, hipMemcpyHostToDevice,
                                 P->stream));
    }
    RF_HIP(P, hipStreamSynchronize(P->stream));
    // diagonal fast path: exactly one stored entry per row, on the diagonal
    bool diag = (M->nnz == M->n);
    for (int32_t i = 0; diag && i < M->n; ++i)
        diag = (M->rowptr[i + 1] - M->rowptr[i] == 1) && (M->colind[M->rowptr[i]] == i);
    D.diagonal = diag;
    if (diag) D.dval = D.val;
    return RF_OK;
}

}  // namespace

// Device-to-host reads through the plan's pinned staging buffer: read() enqueues an
// asynchronous copy on the stream, sync() waits for the stream once and copies every
// pending read out.  (A copy into pageable memory would wait for the stream by
// itself, once per array.)  Use in straight-line code: nothing that syncs another
// Readback of the same plan may run between read() and sync().
struct Readback {
    rf_plan *P;
    hipStream_t s;
    size_t off = 0;
    struct Item { void *dst; size_t off, bytes; };
    std::vector<Item> items;
    Readback(rf_plan *p, hipStream_t st) : P(p), s(st) {}
    hipError_t read(void *dst, const void *src, size_t bytes) {
        const size_t o = (off + 63) & ~size_t(63);
        if (!P->h_stage || o + bytes > P->stage_bytes)
            return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
        hipError_t e = hipMemcpyAsync(P->h_stage + o, src, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) {
            items.push_back({dst, o, bytes});
            off = o + bytes;
        }
        return e;
    }
    // one copy of a device block, handed out in parts (destination, byte offset in the
    // block, bytes)
    hipError_t read_parts(const void *src, size_t total,
                          std::initializer_list<std::tuple<void *, size_t, size_t>> parts) {
        const size_t o = (off + 63) & ~size_t(63);
        if (!P->h_stage || o + total > P->stage_bytes) {
            for (const auto &pt : parts) {
                hipError_t e = hipMemcpyAsync(std::get<0>(pt), static_cast<const char *>(src) + std::get<1>(pt),
                                              std::get<2>(pt), hipMemcpyDeviceToHost, s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        hipError_t e = hipMemcpyAsync(P->h_stage + o, src, total, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) {
            for (const auto &pt : parts) items.push_back({std::get<0>(pt), o + std::get<1>(pt), std::get<2>(pt)});
            off = o + total;
        }
        return e;
    }
    hipError_t sync() {
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            for (const Item &it : items) std::memcpy(it.dst, P->h_stage + it.off, it.bytes);
        items.clear();
        off = 0;
        return e;
    }
};

rf_status rf_fail(rf_plan *plan, rf_status s, const std::string &msg) {
    if (plan) plan->last_error = msg;
    return s;
}

// After the plan's stream has drained: did a cluster solve launched since the last check
// give up a wait or run a member off its XCD?  Either voids that launch's results; the
// plan then keeps to the per-slice solves.
static rf_status cluster_check(rf_plan *P) {
    if (!P->F.cerr || P->F.cepoch == P->F.cerr_seen) return RF_OK;
    unsigned h[2] = {0, 0};
    RF_HIP(P, hipMemcpyAsync(h, P->F.cerr, sizeof(h), hipMemcpyDeviceToHost, P->stream));
    RF_HIP(P, hipStreamSynchronize(P->stream));
    const unsigned seen = P->F.cerr_seen;
    P->F.cerr_seen = P->F.cepoch;
    if (h[0] > seen || h[1] > seen) {
        P->F.cluster_ok = false;
        return rf_fail(P, RF_ERR_DEVICE, h[1] > seen
                       ? "band solve: more cluster workgroups ran on one XCD than its share of the grid"
                       : "band solve: a cluster handoff wait timed out");
    }
    return RF_OK;
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
    o->q_max = 0;
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
    if (plan->fac_graph) (void)hipGraphExecDestroy(plan->fac_graph);
    plan->prof.release();
    for (void *p : plan->allocations) {
        if (plan->alloc.alloc) plan->alloc.free(p, plan->alloc.ctx);
        else (void)hipFree(p);
    }
    if (plan->h_pinned_int) (void)hipHostFree(plan->h_pinned_int);
    if (plan->h_stage) (void)hipHostFree(plan->h_stage);
    delete plan;
}

}  // extern "C"

namespace {

// Plan creation.  owner != null: the plan's band factors live in owner's storage,
// starting at pole `pole_offset` (batched disks); poles != null: factor exactly these
// poles instead of the disk's trapezoidal nodes (the batch's factor owner).
rf_status plan_create_impl(const rf_csr *A, const rf_csr *B, const rf_opts *opts,
                           const rf_allocator *allocator, void *hip_stream, rf_plan_t *out,
                           const rf_plan *owner, int pole_offset, const std::vector<zd> *poles,
                           const rf_plan *adjoint_of = nullptr) {
    if (!out) return RF_ERR_ARG;
    *out = nullptr;
    if (allocator && (!allocator->alloc || !allocator->free)) return RF_ERR_ARG;
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
    if (o.tile < 0 || o.tile > 256 || (o.tile > 0 && (o.tile < 16 || (o.tile & (o.tile - 1)) != 0)))
        return RF_ERR_ARG;
    if (o.trsm_cols < 0 || o.trsm_cols > 8) return RF_ERR_ARG;
    if (o.q_max < 0 || o.q_max > 256) return RF_ERR_ARG;
    if (o.precision < 0 || o.precision > 1) return RF_ERR_ARG;
    if (o.refine < 0 || o.refine > 4 || (o.refine > 0 && o.precision != 1)) return RF_ERR_ARG;
    if (o.solve_form < 0 || o.solve_form > 1) return RF_ERR_ARG;

    rf_plan *P = new rf_plan();
    if (allocator) P->alloc = *allocator;
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
    for (int k = 0; k < 2; ++k) {
        const rf_csr *M = k ? B : A;
        HostCsr &H = k ? P->hB : P->hA;
        H.n = M->n;
        H.rowptr.assign(M->rowptr, M->rowptr + M->n + 1);
        H.colind.assign(M->colind, M->colind + M->nnz);
        H.val.assign(M->val, M->val + 2 * M->nnz);
    }
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            P->max_lds = lds;
        else
            (void)hipGetLastError();
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            P->num_cu = cus;
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
    if (nb == 0) {
        // tile: the smallest power of two >= max(16, kl, ku)
        nb = 16;
        while (nb < std::max(kl, ku)) nb *= 2;
    }
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
    if (poles) {
        if (int(poles->size()) != o.p) return fail(RF_ERR_ARG);
        P->poles = *poles;
    }
    if (owner && (owner->F.nb != nb || owner->n != P->n || pole_offset < 0 ||
                  pole_offset + o.p > owner->opts.p)) {
        rf_fail(P, RF_ERR_ARG, "disk does not fit the shared factor storage");
        return fail(RF_ERR_ARG);
    }
    outer_rule(o.q, P->shifts, P->oweights, P->oextra);
    const int nq = int(P->shifts.size());
    // least-squares storage covers the largest outer rule the plan may use
    std::vector<zd> sh_max, ow_max;
    double ex_max = 0.0;
    outer_rule(std::max(o.q, o.q_max), sh_max, ow_max, ex_max);
    const int nq_alloc = std::max(nq, int(sh_max.size()));

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
    ALLOC(P->d_shifts, std::max(nq_alloc, 1));
    ALLOC(P->d_oweights, std::max(nq_alloc, 1));
    if (hipMemcpyAsync(P->d_poles, P->poles.data(), sizeof(zd) * o.p, hipMemcpyHostToDevice,
                       P->stream) != hipSuccess ||
        hipMemcpyAsync(P->d_weights, P->weights.data(), sizeof(zd) * o.p, hipMemcpyHostToDevice,
                       P->stream) != hipSuccess ||
        (nq > 0 && hipMemcpyAsync(P->d_shifts, P->shifts.data(), sizeof(zd) * nq,
                                  hipMemcpyHostToDevice, P->stream) != hipSuccess) ||
        (nq > 0 && hipMemcpyAsync(P->d_oweights, P->oweights.data(), sizeof(zd) * nq,
                                  hipMemcpyHostToDevice, P->stream) != hipSuccess) ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
        P->broken = true;
        rf_fail(P, RF_ERR_DEVICE, "copy of the rule coefficients failed");
        return fail(RF_ERR_DEVICE);
    }
    const int64_t te = P->F.tile_elems;
    if (owner) {
        // factors of poles pole_offset .. pole_offset + p - 1 of the owner
        P->shared_factors = true;
        P->F.tiles = owner->F.tiles + int64_t(pole_offset) * P->F.nblk * 5 * te;
        P->F.perm = owner->F.perm + int64_t(pole_offset) * P->F.nblk * 2 * nb;
        P->F.info = owner->F.info + pole_offset;
        if (o.precision == 1) {
            if (!owner->F.tiles32) {
                rf_fail(P, RF_ERR_ARG, "the shared factor storage has no complex64 copy");
                return fail(RF_ERR_ARG);
            }
            P->F.tiles32 = owner->F.tiles32 + int64_t(pole_offset) * P->F.nblk * 5 * te;
        }
        if (owner->F.ftiles && o.precision == 0 && o.solve_form == 0)
            P->F.ftiles = owner->F.ftiles + int64_t(pole_offset) * P->F.nblk * 4 * te;
    } else if (adjoint_of) {
        // conjugate transposes of adjoint_of's factor tiles (made by rf_factor_shifts)
        if (adjoint_of->F.nb != nb || adjoint_of->F.nblk != P->F.nblk || adjoint_of->opts.p != o.p) {
            rf_fail(P, RF_ERR_ARG, "adjoint pencil does not match the plan's band tiles");
            return fail(RF_ERR_ARG);
        }
        if (o.precision != 0) {
            rf_fail(P, RF_ERR_ARG, "the adjoint solves run in complex128 only (precision 0)");
            return fail(RF_ERR_ARG);
        }
        ALLOC(P->F.tiles, int64_t(o.p) * P->F.nblk * 5 * te);
        ALLOC(P->F.perm, int64_t(o.p) * P->F.nblk * 2 * nb);
        ALLOC(P->F.info, o.p);
        P->F.adjoint = true;
        P->adj_parent = adjoint_of;
    } else {
        ALLOC(P->F.tiles, int64_t(o.p) * P->F.nblk * 5 * te);
        ALLOC(P->F.perm, int64_t(o.p) * P->F.nblk * 2 * nb);
        ALLOC(P->F.window, int64_t(o.p) * 2 * (2 * nb) * (3 * nb));   // double-buffered per pole
        ALLOC(P->F.info, o.p);
        ALLOC(P->F.rows, int64_t(o.p) * P->F.nblk * te * 3);
        ALLOC(P->F.subperm, int64_t(o.p) * 2 * nb);
        if (o.precision == 1) ALLOC(P->F.tiles32, int64_t(o.p) * P->F.nblk * 5 * te);
        if (o.precision == 0 && o.solve_form == 0 && cluster_solve_supported(nb))
            ALLOC(P->F.ftiles, int64_t(o.p) * P->F.nblk * 4 * te);
    }
    if (P->F.ftiles) {
        // exchange area, sequence flags and error words of the cluster solve (per plan:
        // the disks of a batch solve on their own streams)
        ALLOC(P->F.xchg, cluster_xchg_elems(nb, P->num_cu));
        ALLOC(P->F.cflags, cluster_flag_words(nb, P->num_cu));
        ALLOC(P->F.cerr, 2);
        ALLOC(P->F.ctickets, 8 * 32);
        if (hipMemsetAsync(P->F.cflags, 0, cluster_flag_words(nb, P->num_cu) * 8, P->stream) != hipSuccess ||
            hipMemsetAsync(P->F.cerr, 0, 2 * sizeof(unsigned), P->stream) != hipSuccess ||
            cluster_gate_init(dev) != hipSuccess) {
            (void)hipGetLastError();
            P->broken = true;
            rf_fail(P, RF_ERR_DEVICE, "cluster solve set-up failed");
            return fail(RF_ERR_DEVICE);
        }
    }
    ALLOC(P->d_colcoef, int64_t(std::max(nq_alloc, 1)) * o.w);
    ALLOC(P->d_colw, int64_t(o.p) * o.w);
    ALLOC(P->d_lam, o.w);
    const int64_t n = P->n, w = o.w;
    ALLOC(P->rhs, npad * w);
    ALLOC(P->ypart, int64_t(o.p) * npad * w);
    ALLOC(P->xpart, int64_t(o.p) * npad * w);
    if (o.refine > 0) ALLOC(P->refres, int64_t(o.p) * npad * w);
    ALLOC(P->ytil, n * w);
    ALLOC(P->tmp, n * w);
    ALLOC(P->Wk, n * w);
    ALLOC(P->Gin, n * w);
    const int64_t mb = int64_t(P->mmax) * b, ldc = int64_t(P->mmax + 1) * b;
    ALLOC(P->V, int64_t(P->nsub) * n * ldc);
    ALLOC(P->Hm, int64_t(P->nsub) * ldc * mb);
    ALLOC(P->R0, int64_t(P->nsub) * b * b);
    const int64_t nqs = int64_t(std::max(nq_alloc, 1)) * P->nsub;
    ALLOC(P->lsQ, nqs * P->mmax * 4 * b * b);
    ALLOC(P->lsR, nqs * mb * mb);
    ALLOC(P->lsG, nqs * ldc * b);
    ALLOC(P->lsWork, nqs * ldc * b);
    ALLOC(P->lsY, nqs * mb * b);
    ALLOC(P->ycomb, int64_t(P->nsub) * mb * b);
    ALLOC(P->resid, nqs * b);
    ALLOC(P->r0norm, int64_t(P->nsub) * b);
    ALLOC(P->colnorm, std::max<int64_t>(w, 1) * 2);
    // small-matrix scratch: CholeskyQR work (<= 6 k^2 per block, batched), the panel
    // Gram-Schmidt coefficients and factor of orth_panels (after a 5*64^2 offset)
    ALLOC(P->small, std::max<int64_t>(8 * w * w, 5 * 64 * 64 + 64 * w + 64 * 64) + 8 * int64_t(P->nsub) * b * b);
    ALLOC(P->hbuf, 2 * int64_t(P->nsub) * ldc * b);
    ALLOC(P->rnew, int64_t(P->nsub) * b * b);
    P->partial_elems = std::max<int64_t>(int64_t(1) << 22, 16 * w * w);
    ALLOC(P->partial, P->partial_elems);
    ALLOC(P->flag, 64 + w);
    // Cholesky flags and diagonal ratios side by side: one read fetches both
    ALLOC(P->d_dratio, 2 * w + (2 * w * int64_t(sizeof(int)) + 7) / 8);
    P->d_status = reinterpret_cast<int *>(P->d_dratio + 2 * w);
    ALLOC(P->d_active, w);
    if (hipHostMalloc(reinterpret_cast<void **>(&P->h_pinned_int), sizeof(int) * w, 0) != hipSuccess) {
        (void)hipGetLastError();
        P->h_pinned_int = nullptr;
        rf_fail(P, RF_ERR_NOMEM, "pinned host allocation failed");
        return fail(RF_ERR_NOMEM);
    }
    {
        // status flags, residuals, column norms and the projected pencil
        const int64_t nqm = std::max<int64_t>(std::max(o.q, o.q_max), 1);
        P->stage_bytes = size_t(2 * w * w) * sizeof(zd) + size_t(nqm * w + 8 * w) * sizeof(double) +
                         (size_t(1) << 16);
        if (hipHostMalloc(reinterpret_cast<void **>(&P->h_stage), P->stage_bytes, 0) != hipSuccess) {
            (void)hipGetLastError();
            P->h_stage = nullptr;
            rf_fail(P, RF_ERR_NOMEM, "pinned host allocation failed");
            return fail(RF_ERR_NOMEM);
        }
    }
    ALLOC(P->hV, n * w);
    ALLOC(P->hAV, n * w);
    ALLOC(P->hBV, n * w);
    ALLOC(P->hW, n * w);
    ALLOC(P->hX, n * w);
    ALLOC(P->hY, n * w);
    if (o.q_max > o.q) {
        ALLOC(P->hV2, n * w);
        ALLOC(P->hAV2, n * w);
        ALLOC(P->hBV2, n * w);
    }
    ALLOC(P->hproj, 2 * w * w);
    ALLOC(P->herr, 2 * w);
#undef ALLOC
    *out = P;
    return RF_OK;
}

}  // namespace

extern "C" {

rf_status rf_plan_create(const rf_csr *A, const rf_csr *B, const rf_opts *opts,
                         const rf_allocator *allocator, void *hip_stream, rf_plan_t *out) {
    return plan_create_impl(A, B, opts, allocator, hip_stream, out, nullptr, 0, nullptr);
}

rf_status rf_factor_shifts(rf_plan_t P) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (P->shared_factors)
        return rf_fail(P, RF_ERR_STATE, "the factors of a batched disk come from rf_batch_factor");
    if (P->adj_parent) {
        // adjoint pencil: K_i^H of the parent's factors, no factorization of its own
        const rf_plan *Q = P->adj_parent;
        if (!Q->F.ready)
            return rf_fail(P, RF_ERR_STATE, "the plan of the adjoint pencil has no factors yet "
                                            "(rf_factor_shifts on it first)");
        P->F.ready = false;
        hipEvent_t ev = nullptr;
        P->prof.record_begin(P->stream, ev);
        RF_HIP(P, launch_tiles_adjoint(*P, *Q, P->stream));
        P->prof.record_end(P->stream, ev, 0, 1);
        RF_HIP(P, hipStreamSynchronize(P->stream));
        P->F.ready = true;
        return RF_OK;
    }
    hipEvent_t ev0 = nullptr;
    P->prof.record_begin(P->stream, ev0);
    if (!P->opts.no_graph && P->stream) {
        // the factorization is a fixed sequence of about 2 nb_steps launches that only
        // depends on the plan's shapes and buffers: record it once, replay it after
        if (!P->fac_graph) {
            hipGraph_t g = nullptr;
            RF_HIP(P, hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
            const hipError_t le = launch_band_factor(*P, P->stream);
            const hipError_t ce = hipStreamEndCapture(P->stream, &g);
            if (le != hipSuccess || ce != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                RF_HIP(P, le != hipSuccess ? le : ce);
            }
            hipGraphExec_t ex = nullptr;
            const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            RF_HIP(P, ie);
            P->fac_graph = ex;
        }
        RF_HIP(P, hipGraphLaunch(P->fac_graph, P->stream));
    } else {
        RF_HIP(P, launch_band_factor(*P, P->stream));
    }
    P->prof.record_end(P->stream, ev0, 0, 1);
    std::vector<int32_t> info(P->opts.p);
    {
        Readback rb(P, P->stream);
        RF_HIP(P, rb.read(info.data(), P->F.info, sizeof(int32_t) * P->opts.p));
        RF_HIP(P, rb.sync());
    }
    for (int i = 0; i < P->opts.p; ++i)
        if (info[i] < 0) {
            P->F.ready = false;
            return rf_fail(P, RF_ERR_DEVICE,
                           "band factorization of pole " + std::to_string(i) +
                               ": a pivot step was not published in time");
        } else if (info[i] != 0) {
            P->F.ready = false;
            return rf_fail(P, RF_ERR_SINGULAR,
                           "zero pivot in the factorization of pole " + std::to_string(i) +
                               " at column " + std::to_string(info[i] - 1));
        }
    if (P->F.tiles32) {
        RF_HIP(P, launch_tiles_to_c64(*P, P->stream));
        RF_HIP(P, hipStreamSynchronize(P->stream));
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
    return cluster_check(P);
}

rf_status rf_apply_inner_noalloc(rf_plan_t P, const void *X, int64_t ldx, int32_t ncols, void *Zp,
                                 int64_t ldz) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!X || !Zp || ncols < 0 || ldx < P->n || ldz < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad block arguments");
    const size_t per = inner_scratch_per_column(*P) + 3 * 256;
    if (per > inner_scratch_capacity())
        return rf_fail(P, RF_ERR_ARG, "one column needs " + std::to_string(per) +
                                          " bytes of work space; the library's static array holds " +
                                          std::to_string(inner_scratch_capacity()));
    if (!P->F.ready) return rf_fail(P, RF_ERR_STATE, "rf_factor_shifts has not succeeded");
    if (ncols == 0) return RF_OK;
    RF_HIP(P, launch_inner_apply_static(*P, static_cast<const zd *>(X), ldx, ncols,
                                        static_cast<zd *>(Zp), ldz, P->stream));
    return RF_OK;
}

namespace {

const double kUnit = 1.1102230246251565e-16;

// Breakdown flags (2 cnt ints) and diagonal ratios (2 cnt doubles) of the batched
// Cholesky passes, from their joint device block in one copy.
hipError_t read_chol_flags(Readback &rb, rf_plan *P, int *st, double *dr, int cnt) {
    const size_t w = size_t(P->opts.w);
    const size_t total = 2 * w * sizeof(double) + 2 * w * sizeof(int);
    return rb.read_parts(P->d_dratio, total,
                         {{dr, 0, sizeof(double) * 2 * cnt}, {st, 2 * w * sizeof(double), sizeof(int) * 2 * cnt}});
}

// Orthonormalise one n x k block Wb (ld n) in place by CholeskyQR2, with a shifted
// first pass (CholeskyQR3) when the Gram matrix is numerically indefinite.  Rout
// (k x k, device, may be null) receives the factor with Wb_in = Q Rout.
// tmp: n x k scratch.  Used for blocks wider than the batched path supports.
rf_status cholqr(rf_plan *P, zd *Wb, int64_t n, int k, zd *Rout, zd *tmp) {
    hipStream_t s = P->stream;
    zd *S = P->small;                      // k x k
    zd *R1 = S + int64_t(k) * k;
    zd *R1i = R1 + int64_t(k) * k;
    zd *R2 = R1i + int64_t(k) * k;
    zd *R2i = R2 + int64_t(k) * k;
    zd *Racc = R2i + int64_t(k) * k;
    int *status = P->d_status;
    double *dratio = P->d_dratio;
    int passes = 1;
    for (int attempt = 0; attempt < 2; ++attempt) {
        double shift = attempt == 0 ? 0.0 : 11.0 * (double(n) * k + double(k) * (k + 1)) * kUnit;
        RF_HIP(P, launch_gemm_cn(n, k, k, Z(1), Wb, n, 0, Wb, n, 0, Z(0), S, k, 0, 1, P->partial,
                                 P->partial_elems, s));
        RF_HIP(P, launch_chol_inv(k, S, 0, R1, 0, R1i, 0, 1, status, dratio, shift, s));
        int hstat = 0;
        double dr = 0.0;
        Readback rb(P, s);
        RF_HIP(P, rb.read(&hstat, status, sizeof(int)));
        RF_HIP(P, rb.read(&dr, dratio, sizeof(double)));
        RF_HIP(P, rb.sync());
        if (hstat == 0) { passes = (attempt == 0 && dr > 1e-5) ? 1 : 2; break; }
        if (attempt == 1) return rf_fail(P, RF_ERR_NOCONV, "CholeskyQR breakdown (rank-deficient block)");
    }
    RF_HIP(P, launch_gemm_nn(n, k, k, Z(1), Wb, n, 0, R1i, k, 0, Z(0), tmp, n, 0, 1, s));
    RF_HIP(P, hipMemcpyAsync(Racc, R1, sizeof(zd) * k * k, hipMemcpyDeviceToDevice, s));
    zd *src = tmp, *dst = Wb;
    for (int pass = 0; pass < passes; ++pass) {
        RF_HIP(P, launch_gemm_cn(n, k, k, Z(1), src, n, 0, src, n, 0, Z(0), S, k, 0, 1, P->partial,
                                 P->partial_elems, s));
        RF_HIP(P, launch_chol_inv(k, S, 0, R2, 0, R2i, 0, 1, status, dratio, 0.0, s));
        RF_HIP(P, launch_gemm_nn(n, k, k, Z(1), src, n, 0, R2i, k, 0, Z(0), dst, n, 0, 1, s));
        RF_HIP(P, launch_gemm_nn(k, k, k, Z(1), R2, k, 0, Racc, k, 0, Z(0), R1, k, 0, 1, s));
        RF_HIP(P, hipMemcpyAsync(Racc, R1, sizeof(zd) * k * k, hipMemcpyDeviceToDevice, s));
        std::swap(src, dst);
    }
    if (src != Wb) RF_HIP(P, hipMemcpyAsync(Wb, src, sizeof(zd) * n * k, hipMemcpyDeviceToDevice, s));
    if (Rout) RF_HIP(P, hipMemcpyAsync(Rout, Racc, sizeof(zd) * k * k, hipMemcpyDeviceToDevice, s));
    int hstat = 0;
    {
        Readback rb(P, s);
        RF_HIP(P, rb.read(&hstat, status, sizeof(int)));
        RF_HIP(P, rb.sync());
    }
    if (hstat != 0) return rf_fail(P, RF_ERR_NOCONV, "CholeskyQR breakdown in the second pass");
    return RF_OK;
}

// Batched CholeskyQR2 of `batch` blocks W_t = W + t sW (n x k, ld n, k <= 64), in
// place; R_t (k x k) goes to R + t k^2.  Enqueued only: the caller reads the
// breakdown flags (d_status, two passes) and condition estimates (d_dratio) at its
// next synchronisation and redoes flagged blocks with cholqr().  tmp: n x k x batch.
rf_status cholqr2_batched_enqueue(rf_plan *P, zd *W, int64_t sW, int batch, int64_t n, int k,
                                  zd *R, zd *tmp) {
    hipStream_t s = P->stream;
    const int64_t kk = int64_t(k) * k;
    zd *S = P->small;                      // batch x k x k each
    zd *R1 = S + batch * kk, *R1i = R1 + batch * kk, *R2 = R1i + batch * kk, *R2i = R2 + batch * kk;
    RF_HIP(P, launch_gemm_cn(n, k, k, Z(1), W, n, sW, W, n, sW, Z(0), S, k, kk, batch, P->partial,
                             P->partial_elems, s));
    RF_HIP(P, launch_chol_inv(k, S, kk, R1, kk, R1i, kk, batch, P->d_status, P->d_dratio, 0.0, s));
    RF_HIP(P, launch_gemm_nn(n, k, k, Z(1), W, n, sW, R1i, k, kk, Z(0), tmp, n, n * k, batch, s));
    RF_HIP(P, launch_gemm_cn(n, k, k, Z(1), tmp, n, n * k, tmp, n, n * k, Z(0), S, k, kk, batch,
                             P->partial, P->partial_elems, s));
    RF_HIP(P, launch_chol_inv(k, S, kk, R2, kk, R2i, kk, batch, P->d_status + batch,
                              P->d_dratio + batch, 0.0, s));
    RF_HIP(P, launch_gemm_nn(n, k, k, Z(1), tmp, n, n * k, R2i, k, kk, Z(0), W, n, sW, batch, s));
    RF_HIP(P, launch_gemm_nn(k, k, k, Z(1), R2, k, kk, R1, k, kk, Z(0), R, k, kk, batch, s));
    return RF_OK;
}

// Read the flags of cholqr2_batched_enqueue (after a synchronisation) and redo the
// blocks that broke down or were too ill-conditioned for two passes, from `backup`
// (same layout as W), with the robust single-block routine.  A block that is
// (numerically) rank deficient has orthonormal columns that are arbitrary in the
// deficient directions; when `basis` is given (the Krylov basis the block must stay
// orthogonal to: basis[t], n x kb) those columns are projected off the basis twice
// and re-orthonormalised.  The factor R is kept: its columns for the deficient
// directions are tiny, so the Arnoldi relation changes only by rounding-level terms.
rf_status cholqr2_batched_fixup(rf_plan *P, zd *W, int64_t sW, const zd *backup, int64_t sB,
                                int batch, int64_t n, int k, zd *R, zd *tmp,
                                const std::vector<int> &st, const std::vector<double> &dr,
                                const std::vector<const zd *> *basis = nullptr, int kb = 0) {
    hipStream_t s = P->stream;
    for (int t = 0; t < batch; ++t) {
        bool bad = st[t] != 0 || st[batch + t] != 0 || !(dr[t] > 1e-6);
        if (!bad) continue;
        zd *Wt = W + t * sW;
        RF_HIP(P, launch_copy_cols(n, k, backup + t * sB, n, Wt, n, s));
        RF_TRY(cholqr(P, Wt, n, k, R + int64_t(t) * k * k, tmp));
        if (basis && kb > 0) {
            const zd *Vt = (*basis)[t];
            zd *h = P->hbuf;             // kb x k coefficients (free at this point of a step)
            for (int pass = 0; pass < 2; ++pass) {
                RF_HIP(P, launch_gemm_cn(n, kb, k, Z(1), Vt, n, 0, Wt, n, 0, Z(0), h, kb, 0, 1,
                                         P->partial, P->partial_elems, s));
                RF_HIP(P, launch_gemm_nn(n, kb, k, Z(-1), Vt, n, 0, h, kb, 0, Z(1), Wt, n, 0, 1, s));
            }
            zd *Rdiscard = P->small + 7 * int64_t(k) * k;
            RF_TRY(cholqr(P, Wt, n, k, Rdiscard, tmp));
        }
    }
    return RF_OK;
}

// Block multi-shift GMRES on w/b independent sub-blocks of width b, each with its own
// block-Arnoldi basis of G; the basis of Ytilde = G(Y) is shared by every shift
// (the shift invariance of the Krylov space, Sec. 3.2).  The work is split so that
// the basis can outlive one outer rule (Alg. composite2):
//   krylov_start    Ytilde = G(Y), unit columns, first basis block;
//   krylov_rule     install an outer rule: E1 R0 right-hand sides and the least
//                   squares of every shift replayed over the existing depth;
//   krylov_advance  block-Arnoldi steps until every column of every sub-block meets
//                   the tolerance for every shift;
//   krylov_combine  U = sum_j c'_j (G - s_j I)^{-1} Ytilde (+ (1/q) Ytilde, odd q).
struct KrylovState {
    std::function<bool()> poll;  // optional: called after every block step; true stops the process
    bool stopped = false;        // the poll stopped it (the basis is incomplete)
    std::vector<int> msteps;   // basis depth (blocks) per sub-block
    std::vector<double> scale; // column norms of Ytilde
    int64_t inner_cols = 0;
    int steps = 0;
    double worst = 0.0;
    bool converged = true;
};

// RFEIG_TRACE=1 in the environment: one line per sweep on stderr.
bool trace_on() {
    static const bool on = [] {
        const char *v = std::getenv("RFEIG_TRACE");
        return v && *v && *v != '0';
    }();
    return on;
}

// Outer-solve tolerance: the plan's, or at least 1e-6 when the band solves run in
// complex64 (their rounding bounds how far the outer residual can usefully go).
double outer_tol(const rf_plan *P) {
    return P->opts.precision == 1 ? std::max(P->opts.gmres_tol, 1e-6) : P->opts.gmres_tol;
}

rf_status krylov_start_rhs(rf_plan *P, KrylovState &K);

rf_status krylov_start(rf_plan *P, const zd *Y, int64_t ldy, KrylovState &K) {
    std::function<bool()> poll = std::move(K.poll);
    K = KrylovState();
    K.poll = std::move(poll);
    // Ytilde = G(Y)
    RF_HIP(P, launch_inner_apply(*P, Y, ldy, P->opts.w, P->ytil, P->n, P->stream));
    K.inner_cols += P->opts.w;
    return krylov_start_rhs(P, K);
}

// The right-hand side block of the outer solves is in P->ytil: unit columns and the
// first basis block of every sub-block.
rf_status krylov_start_rhs(rf_plan *P, KrylovState &K) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w, b = P->b, nsub = P->nsub, mmax = P->mmax;
    const int64_t ldc = int64_t(mmax + 1) * b;
    const int64_t vstride = n * ldc;
    K.msteps.assign(nsub, 0);
    // The outer solves are column-wise linear in Ytilde: solve for unit-norm
    // columns (so every column meets the relative tolerance on its own scale,
    // whatever the spread of |R_p(lambda)| across the block) and scale back.
    double *d_scale = P->colnorm;          // w column norms
    double *d_inv = P->colnorm + w;        // w inverse norms
    RF_HIP(P, launch_colnorms(n, w, P->ytil, n, nullptr, 0, nullptr, d_scale, s));
    std::vector<double> ones(w, 1.0);
    K.scale.resize(w);
    Readback rb(P, s);
    RF_HIP(P, rb.read(K.scale.data(), d_scale, sizeof(double) * w));     // used after the loop
    RF_HIP(P, launch_inv_pos(w, d_scale, d_inv, 0.0, s));
    RF_HIP(P, hipMemcpyAsync(P->r0norm, ones.data(), sizeof(double) * w, hipMemcpyHostToDevice, s));
    // V_sb[0] R0_sb = Ytilde_sb D_sb^{-1}   (all sub-blocks at once)
    RF_HIP(P, launch_copy_block(n, b, P->ytil, n, n * b, P->V, n, vstride, nsub, s));
    for (int sb = 0; sb < nsub; ++sb)
        RF_HIP(P, launch_scale_cols(n, b, P->V + sb * vstride, n, d_inv + int64_t(sb) * b, s));
    RF_HIP(P, launch_copy_block(n, b, P->V, n, vstride, P->Gin, n, n * b, nsub, s));   // backup
    RF_TRY(cholqr2_batched_enqueue(P, P->V, vstride, nsub, n, b, P->R0, P->tmp));
    std::vector<int> st(2 * nsub);
    std::vector<double> dr(2 * nsub);
    RF_HIP(P, read_chol_flags(rb, P, st.data(), dr.data(), nsub));
    RF_HIP(P, rb.sync());
    RF_TRY(cholqr2_batched_fixup(P, P->V, vstride, P->Gin, n * b, nsub, n, b, P->R0, P->tmp, st, dr));
    return RF_OK;
}

// worst residual of sub-block sb over all shifts and columns (host copy)
double krylov_worst(const rf_plan *P, const std::vector<double> &resid, int sb) {
    const int nq = int(P->shifts.size()), nsub = P->nsub, b = P->b;
    double worst = 0.0;
    for (int l = 0; l < nq; ++l)
        for (int c = 0; c < b; ++c) worst = std::max(worst, resid[(size_t(l) * nsub + sb) * b + c]);
    return worst;
}

// Install the plan's current outer rule (P->shifts / P->oweights) on the existing
// basis: right-hand sides E1 R0 and the least squares replayed step by step.
// `open` gets the sub-blocks that do not yet meet the tolerance for every shift.
rf_status krylov_rule(rf_plan *P, KrylovState &K, std::vector<int> &open) {
    hipStream_t s = P->stream;
    const int b = P->b, nsub = P->nsub, mmax = P->mmax;
    const int nq = int(P->shifts.size());
    const int64_t ldc = int64_t(mmax + 1) * b, bb = int64_t(b) * b;
    open.clear();
    if (nq == 0) return RF_OK;              // q = 1: the filter is (1/q) G(Y) only
    RF_HIP(P, hipMemcpyAsync(P->d_shifts, P->shifts.data(), sizeof(zd) * nq, hipMemcpyHostToDevice, s));
    RF_HIP(P, hipMemcpyAsync(P->d_oweights, P->oweights.data(), sizeof(zd) * nq, hipMemcpyHostToDevice, s));
    RF_HIP(P, hipMemsetAsync(P->lsG, 0, sizeof(zd) * int64_t(nq) * nsub * ldc * b, s));
    for (int l = 0; l < nq; ++l)
        RF_HIP(P, launch_copy_block(b, b, P->R0, b, bb, P->lsG + int64_t(l) * nsub * ldc * b, ldc,
                                    ldc * b, nsub, s));
    int depth = 0;
    for (int sb = 0; sb < nsub; ++sb) depth = std::max(depth, K.msteps[sb]);
    int *h_active = P->h_pinned_int;
    for (int j = 0; j < depth; ++j) {
        int nact = 0;
        for (int sb = 0; sb < nsub; ++sb)
            if (K.msteps[sb] > j) h_active[nact++] = sb;
        RF_HIP(P, hipMemcpyAsync(P->d_active, h_active, sizeof(int) * nact, hipMemcpyHostToDevice, s));
        RF_HIP(P, launch_ls_update(*P, j, P->d_active, nact, s));
        RF_HIP(P, hipStreamSynchronize(s));    // h_active is reused by the next step
    }
    std::vector<double> resid(size_t(nq) * nsub * b);
    if (depth > 0) {
        Readback rb(P, s);
        RF_HIP(P, rb.read(resid.data(), P->resid, sizeof(double) * nq * nsub * b));
        RF_HIP(P, rb.sync());
    }
    for (int sb = 0; sb < nsub; ++sb)
        if (K.msteps[sb] == 0 || !(krylov_worst(P, resid, sb) <= outer_tol(P))) open.push_back(sb);
    return RF_OK;
}

// Block-Arnoldi steps for the sub-blocks in `active` until each meets the tolerance.
// uniform: every sub-block of `active` keeps stepping until all of them meet it
// (their depths stay equal, as the adaptive form needs); otherwise each stops on
// its own.  The sub-blocks of `active` must all be at the same depth.
rf_status krylov_advance(rf_plan *P, KrylovState &K, std::vector<int> active, bool uniform) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int b = P->b, nsub = P->nsub, mmax = P->mmax;
    const int nq = int(P->shifts.size());
    const int64_t ldc = int64_t(mmax + 1) * b, mbmax = int64_t(mmax) * b;
    const int64_t vstride = n * ldc;
    const int64_t hstride = ldc * mbmax;
    const int64_t bb = int64_t(b) * b;
    int *d_active = P->d_active;
    int *h_active = P->h_pinned_int;                 // pinned host mirror of d_active
    std::vector<double> resid(size_t(std::max(nq, 1)) * nsub * b);
    std::vector<int> st(2 * nsub);
    std::vector<double> dr(2 * nsub);
    if (nq == 0) active.clear();
    zd *h1 = P->hbuf;                    // nsub x ((mmax+1)b x b), by active position
    zd *h2 = P->hbuf + int64_t(nsub) * ldc * b;
    zd *Rn = P->rnew;                    // nsub x (b x b)
    int j0 = active.empty() ? 0 : K.msteps[active[0]];
    std::vector<int> uploaded;           // the list last copied to d_active
    for (int j = j0; j < mmax && !active.empty(); ++j) {
        const int nact = int(active.size());
        const int kb = (j + 1) * b;
        if (active != uploaded) {         // the device list changes only when a sub-block stops
            for (int a = 0; a < nact; ++a) h_active[a] = active[a];
            RF_HIP(P, hipMemcpyAsync(d_active, h_active, sizeof(int) * nact, hipMemcpyHostToDevice, s));
            uploaded = active;
        }
        // gather the newest basis block of every active sub-block, apply G
        RF_HIP(P, launch_copy_block(n, b, P->V + int64_t(j) * b * n, n, vstride, P->Gin, n, n * b,
                                    nact, s, d_active, kMapA));
        RF_HIP(P, launch_inner_apply(*P, P->Gin, n, nact * b, P->Wk, n, s));
        K.inner_cols += int64_t(nact) * b;
        // block classical Gram-Schmidt, twice: h = V^H W; W -= V h
        zd *hp[2] = {h1, h2};
        for (int pass = 0; pass < 2; ++pass) {
            RF_HIP(P, launch_gemm_cn(n, kb, b, Z(1), P->V, n, vstride, P->Wk, n, n * b, Z(0), hp[pass],
                                     kb, ldc * b, nact, P->partial, P->partial_elems, s, d_active,
                                     kMapA));
            RF_HIP(P, launch_gemm_nn(n, kb, b, Z(-1), P->V, n, vstride, hp[pass], kb, ldc * b, Z(1),
                                     P->Wk, n, n * b, nact, s, d_active, kMapA));
        }
        // H[sb][0:kb, jb:(j+1)b] = h1 + h2
        zd *Hcol = P->Hm + int64_t(j) * b * ldc;
        RF_HIP(P, launch_copy_block(kb, b, h1, kb, ldc * b, Hcol, ldc, hstride, nact, s, d_active, kMapC));
        RF_HIP(P, launch_add_block(kb, b, Z(1), h2, kb, ldc * b, Hcol, ldc, hstride, nact, s, d_active,
                                   kMapC));
        // V_{j+1} R = W  (backup of W in Gin for the rare fallback)
        RF_HIP(P, launch_copy_cols(n, nact * b, P->Wk, n, P->Gin, n, s));
        RF_TRY(cholqr2_batched_enqueue(P, P->Wk, n * b, nact, n, b, Rn, P->tmp));
        // the fallback check needs the flags before V and H are written
        {
            Readback rb(P, s);
            RF_HIP(P, read_chol_flags(rb, P, st.data(), dr.data(), nact));
            RF_HIP(P, rb.sync());
        }
        {
            std::vector<const zd *> basis(nact);
            for (int a = 0; a < nact; ++a) basis[a] = P->V + active[a] * vstride;
            RF_TRY(cholqr2_batched_fixup(P, P->Wk, n * b, P->Gin, n * b, nact, n, b, Rn, P->tmp, st,
                                         dr, &basis, kb));
        }
        RF_HIP(P, launch_copy_block(n, b, P->Wk, n, n * b, P->V + int64_t(j + 1) * b * n, n, vstride,
                                    nact, s, d_active, kMapC));
        RF_HIP(P, launch_copy_block(b, b, Rn, b, bb, Hcol + int64_t(j + 1) * b, ldc, hstride, nact, s,
                                    d_active, kMapC));
        // per-shift least squares update and residuals
        RF_HIP(P, launch_ls_update(*P, j, d_active, nact, s));
        {
            Readback rb(P, s);
            RF_HIP(P, rb.read(resid.data(), P->resid, sizeof(double) * nq * nsub * b));
            RF_HIP(P, rb.sync());
        }
        K.steps = std::max(K.steps, j + 1);
        std::vector<int> still;
        bool any_open = false;
        for (int sb : active) {
            K.msteps[sb] = j + 1;
            if (!(krylov_worst(P, resid, sb) <= outer_tol(P))) any_open = true;
        }
        for (int sb : active) {
            const double worst = krylov_worst(P, resid, sb);
            const bool open = uniform ? any_open : !(worst <= outer_tol(P));
            if (open && j + 1 < mmax) still.push_back(sb);
            else {
                if (!(worst <= outer_tol(P))) K.converged = false;
                K.worst = std::max(K.worst, worst);
            }
        }
        active.swap(still);
        if (K.poll && !active.empty() && K.poll()) {
            K.stopped = true;
            break;
        }
    }
    return RF_OK;
}

// solve the triangular systems, combine shifts, U_sb = V_sb Ycomb_sb D_sb
rf_status krylov_combine(rf_plan *P, KrylovState &K, zd *U, int64_t ldu) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int b = P->b, nsub = P->nsub, mmax = P->mmax;
    const int64_t ldc = int64_t(mmax + 1) * b, mbmax = int64_t(mmax) * b;
    const int64_t vstride = n * ldc;
    const double *d_scale = P->colnorm;
    int *h_active = P->h_pinned_int;
    RF_HIP(P, hipMemcpyAsync(P->colnorm, K.scale.data(), sizeof(double) * P->opts.w,
                             hipMemcpyHostToDevice, s));
    for (int sb = 0; sb < nsub; ++sb) {
        const int m = K.msteps[sb];
        zd *Us = U + int64_t(sb) * b * ldu;
        if (m == 0 || P->shifts.empty()) {
            RF_HIP(P, hipMemset2DAsync(Us, ldu * sizeof(zd), 0, n * sizeof(zd), b, s));
        } else {
            h_active[sb] = sb;
            RF_HIP(P, hipMemcpyAsync(P->d_active + sb, h_active + sb, sizeof(int), hipMemcpyHostToDevice, s));
            RF_HIP(P, launch_ls_solve(*P, m, P->d_active + sb, 1, s));
            RF_HIP(P, launch_gemm_nn(n, m * b, b, Z(1), P->V + sb * vstride, n, 0,
                                     P->ycomb + int64_t(sb) * mbmax * b, mbmax, 0, Z(0), Us, ldu, 0, 1,
                                     s));
            RF_HIP(P, launch_scale_cols(n, b, Us, ldu, d_scale + int64_t(sb) * b, s));
        }
        if (P->oextra != 0.0)
            RF_HIP(P, launch_axpby_cols(n, b, Z(1), Us, ldu, Z(P->oextra), P->ytil + int64_t(sb) * b * n,
                                        n, Us, ldu, s));
    }
    RF_HIP(P, hipStreamSynchronize(s));
    return cluster_check(P);
}

// U = sum_j c'_j (G - s_j I)^{-1} G(Y) (Alg. composite's filter): a fresh basis,
// every sub-block stopping on its own.
rf_status filter_core(rf_plan *P, const zd *Y, int64_t ldy, zd *U, int64_t ldu,
                      rf_filter_info *info, std::function<bool()> poll = nullptr,
                      bool *stopped = nullptr) {
    const double t0 = now_ms();
    KrylovState K;
    K.poll = std::move(poll);
    RF_TRY(krylov_start(P, Y, ldy, K));
    std::vector<int> open;
    RF_TRY(krylov_rule(P, K, open));
    RF_TRY(krylov_advance(P, K, open, false));
    if (stopped) *stopped = K.stopped;
    if (K.stopped) return RF_OK;
    RF_TRY(krylov_combine(P, K, U, ldu));
    if (info) {
        info->krylov_steps = K.steps;
        info->converged = K.converged ? 1 : 0;
        info->max_residual = K.worst;
        info->inner_columns = K.inner_cols;
        info->ms_total = now_ms() - t0;
    }
    return K.converged ? RF_OK : RF_ERR_NOCONV;
}

// The composite filter applied to a block X with shifts lam (one per column) through
// the residual R = A X - B X diag(lam), for the precision form.  For any column x
// with shift l (exact algebra, no approximation):
//   K_i^{-1} B x = x / (p_i - l) + K_i^{-1} r / (p_i - l)            (K_i = p_i B - A)
//   G x = g x + rho,  g = sum_i w_i / (p_i - l),  rho = sum_i w_i K_i^{-1} r / (p_i - l)
//   (G - s_j)^{-1} G x = g / (g - s_j) x - s_j / (g - s_j) (G - s_j)^{-1} rho,
// so U = sum_j c'_j (G - s_j)^{-1} G X (+ (1/q) G X, odd q; Thm. Rcrm, eq. linearsolve2)
//      = X diag(f(g)) - sum_j c'_j s_j Z_j diag(1 / (g - s_j)) (+ (1/q) rho),
//   f(g) = sum_j c'_j g / (g - s_j) (+ g / q),   Z_j = (G - s_j)^{-1} rho.
// Only rho and the outer solves with right-hand side rho use the band solves, so
// their complex64 rounding is relative to the residual, which shrinks as the Ritz
// pairs converge, instead of to X.
rf_status filter_core_residual(rf_plan *P, const zd *X, int64_t ldx,
                               const std::vector<std::complex<double>> &lam_in, zd *U,
                               int64_t ldu, rf_filter_info *info) {
    const double t0 = now_ms();
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w, p = P->opts.p;
    const int nq = int(P->shifts.size());
    const std::complex<double> c(P->opts.c_re, P->opts.c_im);
    // shifts: the Ritz values, unless one is not finite or sits (numerically) on a pole
    // of G or of the outer rule; then the centre (any shift keeps the identity exact)
    std::vector<std::complex<double>> lam(w), gt(w);
    auto gval = [&](std::complex<double> l) {
        std::complex<double> g = 0.0;
        for (int i = 0; i < p; ++i)
            g += std::complex<double>(P->weights[i].x, P->weights[i].y) /
                 (std::complex<double>(P->poles[i].x, P->poles[i].y) - l);
        return g;
    };
    for (int k = 0; k < w; ++k) {
        std::complex<double> l = k < int(lam_in.size()) ? lam_in[k] : c;
        bool ok = std::isfinite(l.real()) && std::isfinite(l.imag());
        for (int i = 0; ok && i < p; ++i)
            ok = std::abs(std::complex<double>(P->poles[i].x, P->poles[i].y) - l) > 1e-3 * P->opts.r;
        std::complex<double> g = ok ? gval(l) : 0.0;
        for (int j = 0; ok && j < nq; ++j)
            ok = std::abs(g - std::complex<double>(P->shifts[j].x, P->shifts[j].y)) > 1e-6;
        if (!ok) { l = c; g = gval(c); }
        lam[k] = l;
        gt[k] = g;
    }
    std::vector<zd> hl(w), colw(size_t(p) * w), coef(size_t(std::max(nq, 1)) * w), alpha(w);
    for (int k = 0; k < w; ++k) {
        hl[k] = Z(lam[k].real(), lam[k].imag());
        for (int i = 0; i < p; ++i) {
            std::complex<double> v = std::complex<double>(P->weights[i].x, P->weights[i].y) /
                                     (std::complex<double>(P->poles[i].x, P->poles[i].y) - lam[k]);
            colw[size_t(i) * w + k] = Z(v.real(), v.imag());
        }
        std::complex<double> f = P->oextra * gt[k];
        for (int j = 0; j < nq; ++j) {
            const std::complex<double> sj(P->shifts[j].x, P->shifts[j].y),
                cj(P->oweights[j].x, P->oweights[j].y);
            f += cj * gt[k] / (gt[k] - sj);
            const std::complex<double> cc = -cj * sj / (gt[k] - sj);
            coef[size_t(j) * w + k] = Z(cc.real(), cc.imag());
        }
        alpha[k] = Z(f.real(), f.imag());
    }
    RF_HIP(P, hipMemcpyAsync(P->d_lam, hl.data(), sizeof(zd) * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, hipMemcpyAsync(P->d_colw, colw.data(), sizeof(zd) * p * w, hipMemcpyHostToDevice, s));
    if (nq > 0)
        RF_HIP(P, hipMemcpyAsync(P->d_colcoef, coef.data(), sizeof(zd) * nq * w, hipMemcpyHostToDevice, s));
    // R = A X - B X diag(lam)  (complex128), then rho = sum_i K_i^{-1} R diag(w_i / (p_i - lam))
    RF_HIP(P, launch_spmm(P->A, w, X, ldx, P->tmp, n, s));
    RF_HIP(P, launch_spmm(P->B, w, X, ldx, P->Wk, n, s));
    RF_HIP(P, launch_sub_diag(n, w, P->tmp, n, P->Wk, n, P->d_lam, P->tmp, n, s));
    RF_HIP(P, launch_inner_apply(*P, P->tmp, n, w, P->ytil, n, s, false, P->d_colw));
    // the host vectors above are pageable: finish their copies before they go away
    RF_HIP(P, hipStreamSynchronize(s));
    KrylovState K;
    K.inner_cols = w;
    RF_TRY(krylov_start_rhs(P, K));
    std::vector<int> open;
    RF_TRY(krylov_rule(P, K, open));
    RF_TRY(krylov_advance(P, K, open, false));
    P->colcoef_on = true;
    rf_status cs = krylov_combine(P, K, U, ldu);
    P->colcoef_on = false;
    RF_TRY(cs);
    // U += X diag(f(g))
    RF_HIP(P, hipMemcpyAsync(P->d_lam, alpha.data(), sizeof(zd) * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_add_diag(n, w, X, ldx, P->d_lam, U, ldu, s));
    RF_HIP(P, hipStreamSynchronize(s));
    if (info) {
        info->krylov_steps = K.steps;
        info->converged = K.converged ? 1 : 0;
        info->max_residual = K.worst;
        info->inner_columns = K.inner_cols;
        info->ms_total = now_ms() - t0;
    }
    return K.converged ? RF_OK : RF_ERR_NOCONV;
}

// RF_ERR_ARG unless every entry of the caller's n x k block (k <= w) is finite: its
// column 2-norms, formed on the device and read back, must all be finite (a column
// whose norm overflows counts as non-finite too).
rf_status check_block_finite(rf_plan *P, const zd *X, int64_t ldx, int k, const char *what) {
    if (k <= 0) return RF_OK;
    std::vector<double> nrm(k);
    Readback rb(P, P->stream);
    RF_HIP(P, launch_colnorms(P->n, k, X, ldx, nullptr, 0, nullptr, P->herr, P->stream));
    RF_HIP(P, rb.read(nrm.data(), P->herr, sizeof(double) * k));
    RF_HIP(P, rb.sync());
    for (int c = 0; c < k; ++c)
        if (!std::isfinite(nrm[c]))
            return rf_fail(P, RF_ERR_ARG, std::string(what) + ": column " + std::to_string(c) +
                                              " has a non-finite entry");
    return RF_OK;
}

}  // namespace

rf_status rf_filter_apply(rf_plan_t P, const void *Y, int64_t ldy, int32_t ncols, void *U,
                          int64_t ldu, rf_filter_info *info) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!P->F.ready) return rf_fail(P, RF_ERR_STATE, "rf_factor_shifts has not succeeded");
    if (!Y || !U || ncols != P->opts.w || ldy < P->n || ldu < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad block arguments (ncols must equal w)");
    RF_TRY(check_block_finite(P, static_cast<const zd *>(Y), ldy, ncols, "Y"));
    return filter_core(P, static_cast<const zd *>(Y), ldy, static_cast<zd *>(U), ldu, info);
}

namespace {

// orth(U) for a wide block (n x w, in place): panels of at most 64 columns, each
// made orthogonal to the previous panels by classical Gram-Schmidt applied twice
// and then orthonormalised by CholeskyQR2 (the Gram matrices of 64-column panels
// are factored in LDS).  Only the orthonormal basis is kept; its span is that of U.
rf_status orth_panels(rf_plan *P, zd *U, int64_t n, int w) {
    hipStream_t s = P->stream;
    const int kp = 64;
    zd *h = P->small + 5 * 64 * 64;                            // (w - kp) x kp scratch
    zd *R = h + int64_t(w) * kp;                               // kp x kp factor (discarded)
    std::vector<int> st(2);
    std::vector<double> dr(2);
    for (int c0 = 0; c0 < w; c0 += kp) {
        const int k = std::min(kp, w - c0);
        zd *Ut = U + int64_t(c0) * n;
        for (int pass = 0; c0 > 0 && pass < 2; ++pass) {
            RF_HIP(P, launch_gemm_cn(n, c0, k, Z(1), U, n, 0, Ut, n, 0, Z(0), h, c0, 0, 1, P->partial,
                                     P->partial_elems, s));
            RF_HIP(P, launch_gemm_nn(n, c0, k, Z(-1), U, n, 0, h, c0, 0, Z(1), Ut, n, 0, 1, s));
        }
        RF_HIP(P, launch_copy_cols(n, k, Ut, n, P->Gin, n, s));
        RF_TRY(cholqr2_batched_enqueue(P, Ut, n * k, 1, n, k, R, P->tmp));
        {
            Readback rb(P, s);
            RF_HIP(P, read_chol_flags(rb, P, st.data(), dr.data(), 1));
            RF_HIP(P, rb.sync());
        }
        RF_TRY(cholqr2_batched_fixup(P, Ut, n * k, P->Gin, n * k, 1, n, k, R, P->tmp, st, dr));
    }
    return RF_OK;
}

// HSRR(A, B, U, sigma) (Sec. 2.1) in three parts, so that the host QZ can run while the
// device does other work:
//   hsrr_project  V = orth(U) (in P->hV), W = orth(AV - sigma BV), the projected pencil
//                 (W^* A V, W^* B V) copied to the host (pr.A, pr.B);
//   pr.run_qz     complex QZ and eigenvectors on the host (no device access);
//   hsrr_finish   Ritz values, unit-norm Ritz vectors X = V (P_R V_R) in P->hX and the
//                 errors e_i (eq. rel-error).  Needs P->hV as hsrr_project left it.
struct Projected {
    int w = 0;
    zd *V = nullptr, *AV = nullptr, *BV = nullptr;   // the basis and its products (device)
    std::vector<zd> A, B, al, be, vr;
    std::complex<double> sigma{0.0, 0.0};             // W = orth(AV - sigma BV)
    int qz_status = 0;
    double qz_ms = 0.0;           // host time of the last QZ (reported by RFEIG_TRACE)
    double lower_rel = 0.0;       // strict lower part of A - sigma B, relative (reported)
    bool swapped = false;         // the QZ ran on (B, A - sigma B)
    QzStats qz_stats{};
    // The eigenpairs of (A, B).  W comes from a QR of AV - sigma BV, so R = A - sigma B =
    // W^* (AV - sigma BV) is upper triangular up to rounding; the pencil (B, R) has the
    // same eigenvectors and the eigenvalues mu = 1 / (lambda - sigma), and its second
    // matrix is already triangular, so its QZ skips the QR of step 1 (and, measured, needs
    // fewer sweeps: 383-415 against 433-459 on the 128 x 128 workload's pencils).  It is
    // used when R's strict lower part is at the rounding level (else the QZ runs on (A, B)).
    void run_qz() {
        typedef std::complex<double> cd;
        const auto t0 = std::chrono::steady_clock::now();
        const cd *Ac = reinterpret_cast<const cd *>(A.data());
        const cd *Bc = reinterpret_cast<const cd *>(B.data());
        std::vector<cd> R(size_t(w) * w);
        double lmax = 0.0, scale = 0.0;
        for (int j = 0; j < w; ++j)
            for (int i = 0; i < w; ++i) {
                const size_t e = i + size_t(j) * w;
                R[e] = Ac[e] - sigma * Bc[e];
                scale = std::max(scale, std::abs(Ac[e]) + std::abs(sigma) * std::abs(Bc[e]));
                if (i > j) lmax = std::max(lmax, std::abs(R[e]));
            }
        lower_rel = scale > 0.0 ? lmax / scale : 0.0;
        // the entries of A and B are sums over the n rows of the blocks, whose rounding
        // is of the order of 1e-14 of the largest entry (observed: 4e-14 .. 9e-14 at
        // n = 16384); a lower part up to 1e-12 of it is treated as rounding
        swapped = scale > 0.0 && std::isfinite(lmax) && lower_rel <= 1e-12;
        if (swapped) {
            std::vector<cd> a2(w), b2(w);
            qz_status = host_qz_eig_ex(w, reinterpret_cast<const double *>(Bc),
                                       reinterpret_cast<const double *>(R.data()), true,
                                       reinterpret_cast<double *>(a2.data()),
                                       reinterpret_cast<double *>(b2.data()),
                                       reinterpret_cast<double *>(vr.data()));
            // mu = a2 / b2, lambda = sigma + b2 / a2 = (sigma a2 + b2) / a2
            for (int i = 0; i < w; ++i) {
                const cd a = sigma * a2[i] + b2[i];
                al[i] = zmake(a.real(), a.imag());
                be[i] = zmake(a2[i].real(), a2[i].imag());
            }
        } else {
            qz_status = host_qz_eig_ex(w, reinterpret_cast<const double *>(Ac),
                                       reinterpret_cast<const double *>(Bc), false,
                                       reinterpret_cast<double *>(al.data()),
                                       reinterpret_cast<double *>(be.data()),
                                       reinterpret_cast<double *>(vr.data()));
        }
        qz_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        qz_stats = host_qz_last_stats;
    }
};

// buf selects one of the plan's two sets of basis buffers (the adaptive solver keeps
// two levels in flight).
rf_status hsrr_project(rf_plan *P, zd *U, Projected &pr, int buf = 0) {
    hipStream_t s = P->stream;
    if (buf == 1 && !P->hV2) return rf_fail(P, RF_ERR_STATE, "second basis buffer not allocated");
    pr.V = buf ? P->hV2 : P->hV;
    pr.AV = buf ? P->hAV2 : P->hAV;
    pr.BV = buf ? P->hBV2 : P->hBV;
    const int64_t n = P->n;
    const int w = P->opts.w;
    const std::complex<double> sigma =
        std::isnan(P->opts.sigma_re) ? std::complex<double>(P->opts.c_re, P->opts.c_im)
                                     : std::complex<double>(P->opts.sigma_re, P->opts.sigma_im);
    // V = orth(U): normalise columns first (span unchanged), then CholeskyQR
    RF_HIP(P, launch_colnorms(n, w, U, n, nullptr, 0, nullptr, P->colnorm + w, s));
    RF_HIP(P, launch_inv_pos(w, P->colnorm + w, P->colnorm, 1.0, s));
    RF_HIP(P, launch_copy_cols(n, w, U, n, pr.V, n, s));
    RF_HIP(P, launch_scale_cols(n, w, pr.V, n, P->colnorm, s));
    RF_TRY(orth_panels(P, pr.V, n, w));
    // AV, BV, W = orth(AV - sigma BV)
    RF_HIP(P, launch_spmm(P->A, w, pr.V, n, pr.AV, n, s));
    RF_HIP(P, launch_spmm(P->B, w, pr.V, n, pr.BV, n, s));
    RF_HIP(P, launch_axpby_cols(n, w, Z(1), pr.AV, n, Z(-sigma.real(), -sigma.imag()), pr.BV, n,
                                P->hW, n, s));
    RF_TRY(orth_panels(P, P->hW, n, w));
    // projected pencil
    zd *Ah = P->hproj, *Bh = P->hproj + int64_t(w) * w;
    RF_HIP(P, launch_gemm_cn(n, w, w, Z(1), P->hW, n, 0, pr.AV, n, 0, Z(0), Ah, w, 0, 1, P->partial,
                             P->partial_elems, s));
    RF_HIP(P, launch_gemm_cn(n, w, w, Z(1), P->hW, n, 0, pr.BV, n, 0, Z(0), Bh, w, 0, 1, P->partial,
                             P->partial_elems, s));
    pr.w = w;
    pr.sigma = sigma;
    pr.A.resize(size_t(w) * w);
    pr.B.resize(size_t(w) * w);
    pr.al.resize(w);
    pr.be.resize(w);
    pr.vr.resize(size_t(w) * w);
    Readback rb(P, s);
    RF_HIP(P, rb.read(pr.A.data(), Ah, sizeof(zd) * w * w));
    RF_HIP(P, rb.read(pr.B.data(), Bh, sizeof(zd) * w * w));
    RF_HIP(P, rb.sync());
    return RF_OK;
}

rf_status hsrr_finish(rf_plan *P, const Projected &pr, std::vector<std::complex<double>> &lam,
                      std::vector<double> &err) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w;
    if (pr.qz_status != 0) return rf_fail(P, RF_ERR_NOCONV, "QZ iteration did not converge");
    lam.resize(w);
    std::vector<zd> dlam(w);
    for (int i = 0; i < w; ++i) {
        std::complex<double> a(pr.al[i].x, pr.al[i].y), bb(pr.be[i].x, pr.be[i].y);
        lam[i] = (std::abs(bb) > 0.0) ? a / bb : std::complex<double>(INFINITY, 0.0);
        dlam[i] = Z(lam[i].real(), lam[i].imag());
    }
    // X = V (P_R V_R), unit columns
    zd *dvr = P->small;
    RF_HIP(P, hipMemcpyAsync(dvr, pr.vr.data(), sizeof(zd) * w * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_gemm_nn(n, w, w, Z(1), pr.V, n, 0, dvr, w, 0, Z(0), P->hX, n, 0, 1, s));
    RF_HIP(P, launch_colnorms(n, w, P->hX, n, nullptr, 0, nullptr, P->colnorm + w, s));
    RF_HIP(P, launch_inv_pos(w, P->colnorm + w, P->colnorm, 1.0, s));
    RF_HIP(P, launch_scale_cols(n, w, P->hX, n, P->colnorm, s));
    // e_i = ||A x - lam B x|| / ((|c| + r) ||B x||)
    zd *dl = P->small + int64_t(w) * w;
    RF_HIP(P, hipMemcpyAsync(dl, dlam.data(), sizeof(zd) * w, hipMemcpyHostToDevice, s));
    RF_HIP(P, launch_spmm(P->A, w, P->hX, n, pr.AV, n, s));
    RF_HIP(P, launch_spmm(P->B, w, P->hX, n, pr.BV, n, s));
    RF_HIP(P, launch_colnorms(n, w, pr.AV, n, pr.BV, n, dl, P->herr, s));
    RF_HIP(P, launch_colnorms(n, w, pr.BV, n, nullptr, 0, nullptr, P->herr + w, s));
    std::vector<double> e2(2 * w);
    {
        Readback rb(P, s);
        RF_HIP(P, rb.read(e2.data(), P->herr, sizeof(double) * 2 * w));
        RF_HIP(P, rb.sync());
    }
    const double scale = std::abs(std::complex<double>(P->opts.c_re, P->opts.c_im)) + P->opts.r;
    err.resize(w);
    for (int i = 0; i < w; ++i) {
        double den = scale * e2[w + i];
        err[i] = (den > 0.0 && std::isfinite(lam[i].real())) ? e2[i] / den : INFINITY;
    }
    return RF_OK;
}

// HSRR in one piece (Ritz values lam, Ritz vectors in P->hX, errors err).
rf_status hsrr(rf_plan *P, zd *U, std::vector<std::complex<double>> &lam,
               std::vector<double> &err) {
    Projected pr;
    RF_TRY(hsrr_project(P, U, pr));
    pr.run_qz();
    return hsrr_finish(P, pr, lam, err);
}

// Copy the last Ritz pairs into the caller's result, converged pairs inside D first.
rf_status fill_result(rf_plan *P, const std::vector<std::complex<double>> &lam,
                      const std::vector<double> &err, const std::vector<int> &flags,
                      rf_result *res) {
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w;
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
    return RF_OK;
}

}  // namespace

rf_status rf_solve_region(rf_plan_t P, const void *Y0, int64_t ldy, rf_result *res) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!res || !res->lambda || !res->X || !res->err || !res->flags || res->ldx < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad result buffers");
    if (Y0 && ldy < P->n) return rf_fail(P, RF_ERR_ARG, "bad start block");
    if (Y0) RF_TRY(check_block_finite(P, static_cast<const zd *>(Y0), ldy, P->opts.w, "Y0"));
    if (!P->F.ready) RF_TRY(rf_factor_shifts(P));
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w;
    zd *Y = P->hX;   // current block (Ritz vectors after the first sweep)
    if (Y0) RF_HIP(P, launch_copy_cols(n, w, static_cast<const zd *>(Y0), ldy, Y, n, s));
    else RF_HIP(P, launch_gaussian(n, w, Y, n, P->opts.seed, s));
    // Y = orth(Y)  (Alg. composite: orthonormal random start)
    RF_TRY(orth_panels(P, Y, n, w));
    const std::complex<double> c(P->opts.c_re, P->opts.c_im);
    const double r = P->opts.r;
    std::vector<std::complex<double>> lam;
    std::vector<double> err;
    int prev = -1, t = 1;
    bool converged = false;
    double ms_filter = 0.0, ms_hsrr = 0.0;
    std::vector<int> flags(w);
    rf_filter_info fi{};
    // the stopping rule of Alg. composite on sweep t's Ritz pairs
    auto stopping_rule = [&](int sweep, double ms_f) {
        int count = 0;
        bool all_small = true;
        for (int i = 0; i < w; ++i) {
            bool inside = std::abs(lam[i] - c) < r;
            bool filt = inside && err[i] < P->opts.tau_g;
            flags[i] = (inside ? 1 : 0) | (filt ? 2 : 0) | (err[i] <= P->opts.tau ? 4 : 0);
            if (filt) { ++count; if (!(err[i] <= P->opts.tau)) all_small = false; }
        }
        if (trace_on()) {
            double emax = 0.0;
            for (int i = 0; i < w; ++i)
                if (flags[i] & 2) emax = std::max(emax, err[i]);
            std::fprintf(stderr, "[rfeig] sweep %d: filtered %d, max filtered e %.3e, krylov steps %d, "
                                 "outer residual %.2e, filter %.1f ms\n",
                         sweep, count, emax, fi.krylov_steps, fi.max_residual, ms_f);
        }
        const bool stop = all_small && (count == prev || (sweep == 1 && P->opts.expected_count >= 0 &&
                                                          count == P->opts.expected_count));
        prev = count;
        return stop;
    };
    auto filter_into_ytil = [&](const zd *Yin, int sweep, std::function<bool()> poll,
                                bool *stopped) -> rf_status {
        const double t1 = now_ms();
        rf_status fs = (P->opts.precision == 1 && sweep > 1)
                           ? filter_core_residual(P, Yin, n, lam, P->hW, n, &fi)
                           : filter_core(P, Yin, n, P->hW, n, &fi, std::move(poll), stopped);
        if (fs != RF_OK && fs != RF_ERR_NOCONV) return fs;
        if (!(stopped && *stopped)) {
            // U out of hW (HSRR reuses it) into ytil
            RF_HIP(P, launch_copy_cols(n, w, P->hW, n, P->ytil, n, s));
            if (sweep <= 16) res->krylov_steps[sweep - 1] = fi.krylov_steps;
        }
        ms_filter += now_ms() - t1;
        return RF_OK;
    };
    if (P->opts.precision == 1) {
        // precision form: the residual form needs the Ritz pairs of the previous sweep
        for (t = 1; t <= P->opts.max_subspace_it; ++t) {
            RF_TRY(filter_into_ytil(Y, t, nullptr, nullptr));
            const double t2 = now_ms();
            RF_TRY(hsrr(P, P->ytil, lam, err));
            ms_hsrr += now_ms() - t2;
            if (stopping_rule(t, 0.0)) { converged = true; break; }
        }
    } else {
        // Sweep t + 1 filters the orthonormal basis V_t of sweep t's HSRR (P->hV) instead of
        // its Ritz vectors X_t = V_t (P_R V_R): the filter is linear, so span(filter(X_t)) =
        // span(filter(V_t)), and HSRR depends on that span only.  This lets the host QZ of
        // sweep t run while the device already filters for sweep t + 1; sweep t's Ritz
        // pairs are finished between two block-Arnoldi steps as soon as the QZ is done,
        // and if they meet the stopping rule the speculative filter is abandoned.
        RF_TRY(filter_into_ytil(Y, 1, nullptr, nullptr));
        Projected pr;
        for (t = 1;; ++t) {
            double t2 = now_ms();
            RF_TRY(hsrr_project(P, P->ytil, pr));
            ms_hsrr += now_ms() - t2;
            std::atomic<bool> qz_done{false};
            std::thread qz;
            // joins the QZ thread on every way out of this sweep, early error returns included
            struct Joiner {
                std::thread &th;
                ~Joiner() { if (th.joinable()) th.join(); }
            } qz_joiner{qz};
            try {
                qz = std::thread([&] { pr.run_qz(); qz_done.store(true, std::memory_order_release); });
            } catch (...) {                    // no thread: run the QZ here
                pr.run_qz();
                qz_done.store(true);
            }
            bool decided = false;
            rf_status fin = RF_OK;
            auto finish = [&]() {
                const double t3 = now_ms();
                if (qz.joinable()) qz.join();
                fin = hsrr_finish(P, pr, lam, err);
                if (trace_on())
                    std::fprintf(stderr, "[rfeig] sweep %d: host QZ %.1f ms (QR %.1f, HT %.1f, QZ %.1f in %d "
                                         "sweeps, vectors %.1f; pencil %s, lower part %.1e)\n",
                                 t, pr.qz_ms, pr.qz_stats.qr_ms, pr.qz_stats.ht_ms, pr.qz_stats.qz_ms,
                                 pr.qz_stats.sweeps, pr.qz_stats.vec_ms,
                                 pr.swapped ? "(B, A - sigma B)" : "(A, B)", pr.lower_rel);
                decided = true;
                ms_hsrr += now_ms() - t3;
                if (fin == RF_OK) converged = stopping_rule(t, 0.0);
                return fin == RF_OK && converged;
            };
            if (t < P->opts.max_subspace_it) {
                RF_HIP(P, launch_copy_cols(n, w, P->hV, n, P->hY, n, s));
                bool stopped = false;
                auto poll = [&]() {
                    if (decided || !qz_done.load(std::memory_order_acquire)) return false;
                    return finish();
                };
                rf_status fs = filter_into_ytil(P->hY, t + 1, poll, &stopped);
                if (!decided) finish();
                if (fs != RF_OK) return fs;
                RF_TRY(fin);
                if (converged) break;
            } else {
                finish();
                RF_TRY(fin);
                break;
            }
        }
    }
    if (t > P->opts.max_subspace_it) t = P->opts.max_subspace_it;
    RF_TRY(fill_result(P, lam, err, flags, res));
    res->sweeps = t;
    res->converged = converged ? 1 : 0;
    res->ms_filter = ms_filter;
    res->ms_hsrr = ms_hsrr;
    return converged ? RF_OK : RF_ERR_NOCONV;
}

rf_status rf_solve_region_adaptive(rf_plan_t P, const void *Y0, int64_t ldy, rf_result *res) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (!res || !res->lambda || !res->X || !res->err || !res->flags || res->ldx < P->n)
        return rf_fail(P, RF_ERR_ARG, "bad result buffers");
    if (Y0 && ldy < P->n) return rf_fail(P, RF_ERR_ARG, "bad start block");
    if (P->opts.q_max < P->opts.q)
        return rf_fail(P, RF_ERR_ARG, "q_max of the plan must be at least q");
    if (P->opts.precision != 0)
        return rf_fail(P, RF_ERR_ARG, "the precision form needs the subspace iteration (rf_solve_region)");
    if (Y0) RF_TRY(check_block_finite(P, static_cast<const zd *>(Y0), ldy, P->opts.w, "Y0"));
    if (!P->F.ready) RF_TRY(rf_factor_shifts(P));
    hipStream_t s = P->stream;
    const int64_t n = P->n;
    const int w = P->opts.w, nsub = P->nsub;
    zd *Y = P->hX;
    if (Y0) RF_HIP(P, launch_copy_cols(n, w, static_cast<const zd *>(Y0), ldy, Y, n, s));
    else RF_HIP(P, launch_gaussian(n, w, Y, n, P->opts.seed, s));
    RF_TRY(orth_panels(P, Y, n, w));
    const std::complex<double> c(P->opts.c_re, P->opts.c_im);
    const double r = P->opts.r;
    double ms_filter = 0.0, ms_hsrr = 0.0;
    double t1 = now_ms();
    KrylovState K;
    RF_TRY(krylov_start(P, Y, n, K));           // Ytilde = G(Y) once; the basis is kept
    ms_filter += now_ms() - t1;
    std::vector<int> all(nsub), open, flags(w);
    std::iota(all.begin(), all.end(), 0);
    std::vector<std::complex<double>> lam;
    std::vector<double> err;
    int prev = -1, t = 0;
    bool converged = false;
    rf_status out = RF_OK;
    // U of level t (k2 = q 2^t) into P->Wk
    auto level_filter = [&](int level) -> rf_status {
        const double ta = now_ms();
        const int k2 = P->opts.q << level;
        outer_rule(k2, P->shifts, P->oweights, P->oextra);
        RF_TRY(krylov_rule(P, K, open));
        if (!open.empty()) RF_TRY(krylov_advance(P, K, all, true));
        RF_TRY(krylov_combine(P, K, P->Wk, n));
        if (level < 16) res->krylov_steps[level] = K.msteps.empty() ? 0 : K.msteps[0];
        ms_filter += now_ms() - ta;
        return RF_OK;
    };
    auto stopping_rule = [&](int level) {
        int count = 0;
        bool all_small = true;
        for (int i = 0; i < w; ++i) {
            bool inside = std::abs(lam[i] - c) < r;
            bool filt = inside && err[i] < P->opts.tau_g;
            flags[i] = (inside ? 1 : 0) | (filt ? 2 : 0) | (err[i] <= P->opts.tau ? 4 : 0);
            if (filt) { ++count; if (!(err[i] <= P->opts.tau)) all_small = false; }
        }
        const bool stop = all_small && (count == prev || (level == 0 && P->opts.expected_count >= 0 &&
                                                          count == P->opts.expected_count));
        prev = count;
        return stop;
    };
    // Levels are pipelined: while the host QZ of level t runs on its own thread, the
    // device computes level t + 1's filter and projection into the second basis set, and
    // level t + 1's QZ starts on another thread; level t is then finished and tested, and
    // a converged level discards the one behind it.
    const int nlevels = [&] { int m = 0; for (int k2 = P->opts.q; k2 <= P->opts.q_max; k2 *= 2) ++m; return m; }();
    struct Flight {
        Projected pr;
        std::thread th;
        void start() {
            try {
                th = std::thread([this] { pr.run_qz(); });
            } catch (...) {
                pr.run_qz();
            }
        }
        void wait() { if (th.joinable()) th.join(); }
        ~Flight() { wait(); }             // never leaves a joinable thread behind
    };
    Flight fl[2];
    out = level_filter(0);
    if (out == RF_OK) {
        const double ta = now_ms();
        out = hsrr_project(P, P->Wk, fl[0].pr, 0);
        ms_hsrr += now_ms() - ta;
    }
    if (out == RF_OK) fl[0].start();
    for (t = 0; out == RF_OK && t < nlevels; ++t) {
        Flight &cur = fl[t % 2], &nxt = fl[(t + 1) % 2];
        const bool ahead = (t + 1 < nlevels) && P->hV2 != nullptr;
        if (ahead) {
            out = level_filter(t + 1);
            if (out == RF_OK) {
                const double ta = now_ms();
                out = hsrr_project(P, P->Wk, nxt.pr, (t + 1) % 2);
                ms_hsrr += now_ms() - ta;
            }
            if (out == RF_OK) nxt.start();
        }
        const double tb = now_ms();
        cur.wait();
        rf_status fin = (out == RF_OK) ? hsrr_finish(P, cur.pr, lam, err) : out;
        ms_hsrr += now_ms() - tb;
        if (fin != RF_OK) { out = fin; nxt.wait(); break; }
        if (stopping_rule(t)) {
            converged = true;
            nxt.wait();
            ++t;
            break;
        }
        if (!ahead && t + 1 < nlevels) {
            // no second basis set: the next level in order
            out = level_filter(t + 1);
            if (out == RF_OK) {
                const double ta = now_ms();
                out = hsrr_project(P, P->Wk, nxt.pr, 0);
                ms_hsrr += now_ms() - ta;
            }
            if (out == RF_OK) nxt.start();
        }
    }
    fl[0].wait();
    fl[1].wait();
    // the plan's own outer rule (q) for later calls
    outer_rule(P->opts.q, P->shifts, P->oweights, P->oextra);
    if (out != RF_OK) return out;
    RF_TRY(fill_result(P, lam, err, flags, res));
    res->sweeps = t;
    res->converged = converged ? 1 : 0;
    res->ms_filter = ms_filter;
    res->ms_hsrr = ms_hsrr;
    return converged ? RF_OK : RF_ERR_NOCONV;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
hipEvent_t KernelProfile::take() {
    if (pool.empty()) {
        if (pending.size() > 1024) (void)drain();
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
}

void KernelProfile::record_begin(hipStream_t s, hipEvent_t &a) {
    a = on ? take() : nullptr;
    if (a) (void)hipEventRecord(a, s);
}

void KernelProfile::record_end(hipStream_t s, hipEvent_t a, int64_t cols, int kind) {
    if (!a) return;
    hipEvent_t b = take();
    if (!b) { pool.push_back(a); return; }
    (void)hipEventRecord(b, s);
    pending.push_back({a, b, cols, kind});
}

hipError_t KernelProfile::drain() {
    for (auto &p : pending) {
        hipError_t e = hipEventSynchronize(p.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return e;
        if (p.kind == 0) {
            stats.solve_launches += 1;
            stats.solve_columns += p.cols;
            stats.solve_ms += ms;
        } else {
            stats.factor_launches += 1;
            stats.factor_ms += ms;
        }
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
    return hipSuccess;
}

void KernelProfile::release() {
    for (auto &p : pending) { pool.push_back(p.a); pool.push_back(p.b); }
    pending.clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

extern "C" {

rf_status rf_profile_enable(rf_plan_t P, int32_t on) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (on) {
        RF_HIP(P, P->prof.drain());
        P->prof.stats = rf_kernel_stats{};
    }
    P->prof.on = on != 0;
    return RF_OK;
}

rf_status rf_profile_read(rf_plan_t P, rf_kernel_stats *out) {
    if (!P || !out) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    RF_HIP(P, hipStreamSynchronize(P->stream));
    RF_HIP(P, P->prof.drain());
    *out = P->prof.stats;
    return RF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form: several disks of one pencil (Sec. 1: regions handled in parallel).
// One factor owner holds the band factors of every disk's poles and factorizes
// them with one launch sequence; each disk is an ordinary plan whose factor
// pointers address its slice of that storage and which runs on a stream of its own.
// ---------------------------------------------------------------------------
struct rf_batch {
    rf_plan *owner = nullptr;
    std::vector<rf_plan *> disks;
    std::vector<hipStream_t> streams;
    std::string last_error;
};

namespace {

rf_status batch_fail(rf_batch *Bt, rf_status s, const std::string &msg) {
    Bt->last_error = msg;
    return s;
}

void batch_free(rf_batch *Bt) {
    for (rf_plan *d : Bt->disks) rf_plan_destroy(d);
    if (Bt->owner) rf_plan_destroy(Bt->owner);
    for (hipStream_t s : Bt->streams) (void)hipStreamDestroy(s);
    delete Bt;
}

}  // namespace

extern "C" {

rf_status rf_batch_create(const rf_csr *A, const rf_csr *B, const rf_opts *opts, int32_t ndisks,
                          const rf_allocator *allocator, void *hip_stream, rf_batch_t *out) {
    if (!out) return RF_ERR_ARG;
    *out = nullptr;
    if (allocator && (!allocator->alloc || !allocator->free)) return RF_ERR_ARG;
    if (!opts || ndisks < 1 || !csr_ok(A) || !csr_ok(B) || A->n != B->n) return RF_ERR_ARG;
    int64_t ptot = 0;
    for (int d = 0; d < ndisks; ++d) {
        if (opts[d].p < 1 || opts[d].tile != opts[0].tile || opts[d].precision != opts[0].precision)
            return RF_ERR_ARG;
        ptot += opts[d].p;
    }
    if (ptot > (int64_t(1) << 20)) return RF_ERR_ARG;
    rf_batch *Bt = new rf_batch();
    auto fail = [&](rf_status s) {
        *out = Bt;  // kept so the caller can read rf_batch_last_error, then destroy
        return s;
    };
    // the owner's poles: every disk's trapezoidal nodes, disk after disk (eq. pwtp)
    std::vector<zd> poles;
    for (int d = 0; d < ndisks; ++d) {
        const rf_opts &o = opts[d];
        for (int i = 1; i <= o.p; ++i) {
            std::complex<double> pole = std::complex<double>(o.c_re, o.c_im) +
                                        o.r * std::polar(1.0, (2.0 * i - 1.0) * kPi / o.p);
            poles.push_back(Z(pole.real(), pole.imag()));
        }
    }
    // the owner only factorizes: one column, one Krylov block
    rf_opts oo = opts[0];
    oo.p = int32_t(ptot);
    oo.q = 1;
    oo.q_max = 0;
    oo.w = 1;
    oo.subblock = 0;
    oo.max_krylov_blocks = 1;
    rf_status st = plan_create_impl(A, B, &oo, allocator, hip_stream, &Bt->owner, nullptr, 0, &poles);
    if (st != RF_OK) {
        return fail(batch_fail(Bt, st, std::string("factor storage: ") +
                                           (Bt->owner ? Bt->owner->last_error : rf_status_str(st))));
    }
    int off = 0;
    for (int d = 0; d < ndisks; ++d) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return fail(batch_fail(Bt, RF_ERR_DEVICE, "stream creation failed"));
        }
        Bt->streams.push_back(s);
        rf_plan *P = nullptr;
        st = plan_create_impl(A, B, &opts[d], allocator, s, &P, Bt->owner, off, nullptr);
        if (P) Bt->disks.push_back(P);
        if (st != RF_OK) {
            return fail(batch_fail(Bt, st, "disk " + std::to_string(d) + ": " +
                                               (P ? P->last_error : std::string(rf_status_str(st)))));
        }
        off += opts[d].p;
    }
    *out = Bt;
    return RF_OK;
}

rf_status rf_batch_factor(rf_batch_t Bt) {
    if (!Bt || !Bt->owner || Bt->disks.empty()) return RF_ERR_ARG;
    for (rf_plan *d : Bt->disks) d->F.ready = false;
    rf_status st = rf_factor_shifts(Bt->owner);
    if (st != RF_OK) {
        std::string msg = Bt->owner->last_error;
        if (st == RF_ERR_SINGULAR) {
            // name the disk of the first singular pole
            std::vector<int32_t> info(Bt->owner->opts.p);
            if (hipMemcpyAsync(info.data(), Bt->owner->F.info, sizeof(int32_t) * info.size(),
                               hipMemcpyDeviceToHost, Bt->owner->stream) == hipSuccess &&
                hipStreamSynchronize(Bt->owner->stream) == hipSuccess) {
                int off = 0;
                for (size_t d = 0; d < Bt->disks.size(); ++d) {
                    bool bad = false;
                    for (int i = 0; i < Bt->disks[d]->opts.p; ++i) bad |= info[off + i] != 0;
                    if (bad) { msg = "disk " + std::to_string(d) + ": " + msg; break; }
                    off += Bt->disks[d]->opts.p;
                }
            } else {
                (void)hipGetLastError();
            }
        }
        return batch_fail(Bt, st, msg);
    }
    // rf_factor_shifts has drained the owner stream: the factors are complete
    for (rf_plan *d : Bt->disks) d->F.ready = true;
    return RF_OK;
}

rf_plan_t rf_batch_plan(rf_batch_t Bt, int32_t d) {
    if (!Bt || d < 0 || d >= int32_t(Bt->disks.size())) return nullptr;
    return Bt->disks[d];
}

int32_t rf_batch_size(rf_batch_t Bt) { return Bt ? int32_t(Bt->disks.size()) : -1; }

}  // extern "C"

namespace {

// rf_solve_region on several plans at once, at most `threads` at a time, each plan on
// the host thread that takes it (its GPU work goes to the plan's own stream).
void solve_many(rf_plan *const *plans, int np, const void *const *Y0, const int64_t *ldy,
                rf_result *res, rf_status *status, int threads, bool factor = false) {
    const int nt = std::max(1, std::min(threads <= 0 ? np : threads, np));
    // An adjoint plan's factors are the conjugate transposes of its parent's: factorize
    // the plans that own factors first, then transpose into the adjoint plans, then solve.
    std::vector<char> skip(size_t(np), 0);
    bool any_adj = false;
    for (int d = 0; d < np; ++d) any_adj |= plans[d]->adj_parent != nullptr;
    if (any_adj) {
        for (int pass = 0; pass < 2; ++pass)
            for (int d = 0; d < np; ++d) {
                if ((pass == 1) != (plans[d]->adj_parent != nullptr)) continue;
                if (!(factor || !plans[d]->F.ready)) continue;
                if (hipSetDevice(plans[d]->device) != hipSuccess) {
                    (void)hipGetLastError();
                    status[d] = RF_ERR_DEVICE;
                    skip[d] = 1;
                    continue;
                }
                status[d] = rf_factor_shifts(plans[d]);
                if (status[d] != RF_OK) skip[d] = 1;
            }
        factor = false;
    }
    std::atomic<int> next{0};
    auto worker = [&]() {
        for (int d; (d = next.fetch_add(1)) < np;) {
            if (skip[d]) continue;
            if (hipSetDevice(plans[d]->device) != hipSuccess) {
                (void)hipGetLastError();
                status[d] = RF_ERR_DEVICE;
                continue;
            }
            if (factor) {
                status[d] = rf_factor_shifts(plans[d]);
                if (status[d] != RF_OK) continue;
            }
            status[d] = rf_solve_region(plans[d], Y0 ? Y0[d] : nullptr, ldy ? ldy[d] : 0, &res[d]);
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(worker);
        } catch (...) {
            break;                               // fewer threads: the others take more plans
        }
    }
    worker();
    for (auto &t : pool) t.join();
}

}  // namespace

extern "C" {

rf_status rf_solve_regions(int32_t count, rf_plan_t *plans, int32_t factor, const void *const *Y0,
                           const int64_t *ldy, rf_result *res, rf_status *status) {
    if (count < 0 || (count > 0 && (!plans || !res || !status))) return RF_ERR_ARG;
    for (int d = 0; d < count; ++d) status[d] = RF_ERR_ARG;
    for (int d = 0; d < count; ++d) {
        if (!plans[d]) return RF_ERR_ARG;
        for (int e = 0; e < d; ++e)
            if (plans[e] == plans[d]) return RF_ERR_ARG;   // one plan, one thread at a time
    }
    solve_many(plans, count, Y0, ldy, res, status, count, factor != 0);
    for (int d = 0; d < count; ++d)
        if (status[d] != RF_OK) return status[d];
    return RF_OK;
}

rf_status rf_batch_solve(rf_batch_t Bt, const void *const *Y0, const int64_t *ldy, rf_result *res,
                         rf_status *status, int32_t threads) {
    if (!Bt || !res || !status || Bt->disks.empty()) return RF_ERR_ARG;
    const int nd = int(Bt->disks.size());
    for (int d = 0; d < nd; ++d) status[d] = RF_ERR_STATE;
    for (rf_plan *d : Bt->disks)
        if (!d->F.ready) return batch_fail(Bt, RF_ERR_STATE, "rf_batch_factor has not succeeded");
    solve_many(Bt->disks.data(), nd, Y0, ldy, res, status, threads);
    for (int d = 0; d < nd; ++d)
        if (status[d] != RF_OK)
            return batch_fail(Bt, status[d], "disk " + std::to_string(d) + ": " +
                                                 Bt->disks[d]->last_error);
    return RF_OK;
}

const char *rf_batch_last_error(rf_batch_t Bt) { return Bt ? Bt->last_error.c_str() : ""; }

int64_t rf_batch_device_bytes(rf_batch_t Bt) {
    if (!Bt) return -1;
    int64_t t = Bt->owner ? Bt->owner->device_bytes : 0;
    for (rf_plan *d : Bt->disks) t += d->device_bytes;
    return t;
}

void rf_batch_destroy(rf_batch_t Bt) {
    if (Bt) batch_free(Bt);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Differentiation form.  For a simple eigenvalue lambda with right vector x and
// left vector y (y^H A = lambda y^H B) the first-order perturbation is
//   d lambda = y^H (dA - lambda dB) x / (y^H B x)
// (textbook perturbation theory, not part of the paper).  The left vectors are the
// right eigenvectors of the adjoint pencil (A^H, B^H) at conj(lambda), found by the
// same filter over the mirrored disk D(conj c, r): its trapezoidal poles are the
// conjugates of the original ones (eq. pwtp: the angle set is symmetric).
// ---------------------------------------------------------------------------
namespace {

void conj_transpose(const HostCsr &M, std::vector<int32_t> &rp, std::vector<int32_t> &ci,
                    std::vector<double> &v) {
    const int32_t n = M.n;
    const int64_t nnz = int64_t(M.colind.size());
    rp.assign(size_t(n) + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) ++rp[size_t(M.colind[e]) + 1];
    for (int32_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    ci.assign(size_t(nnz), 0);
    v.assign(size_t(2 * nnz), 0.0);
    std::vector<int64_t> next(rp.begin(), rp.end() - 1);
    for (int32_t r = 0; r < n; ++r)       // rows in order: columns of the result stay sorted
        for (int64_t e = M.rowptr[r]; e < M.rowptr[r + 1]; ++e) {
            const int64_t t = next[M.colind[e]]++;
            ci[t] = r;
            v[2 * t] = M.val[2 * e];
            v[2 * t + 1] = -M.val[2 * e + 1];
        }
}

}  // namespace

extern "C" {

rf_status rf_plan_create_adjoint(rf_plan_t P, void *hip_stream, rf_plan_t *out) {
    if (!P || !out) return RF_ERR_ARG;
    *out = nullptr;
    std::vector<int32_t> arp, aci, brp, bci;
    std::vector<double> av, bv;
    conj_transpose(P->hA, arp, aci, av);
    conj_transpose(P->hB, brp, bci, bv);
    rf_csr Ah{P->hA.n, int64_t(aci.size()), arp.data(), aci.data(), av.data()};
    rf_csr Bh{P->hB.n, int64_t(bci.size()), brp.data(), bci.data(), bv.data()};
    rf_opts o = P->opts;
    o.c_im = -o.c_im;
    if (!std::isnan(o.sigma_re)) o.sigma_im = -o.sigma_im;
    if (P->F.adjoint || P->shared_factors)
        return rf_fail(P, RF_ERR_ARG, "adjoint plans are made from a plan that owns its factors");
    return plan_create_impl(&Ah, &Bh, &o, P->alloc.alloc ? &P->alloc : nullptr, hip_stream, out,
                            nullptr, 0, nullptr, P);
}

rf_status rf_eig_vjp(rf_plan_t P, int32_t s, const double *lambda, const void *X, int64_t ldx,
                     int32_t s_left, const double *mu, const void *Yl, int64_t ldyl,
                     const double *g, void *gA, void *gB, double *denom, int32_t *pair_out) {
    if (!P) return RF_ERR_ARG;
    if (P->broken) return rf_fail(P, RF_ERR_STATE, "plan is unusable after a device error");
    if (s < 0 || s > P->opts.w || s_left < 0 || (s > 0 && (!lambda || !X || !mu || !Yl || !g || !gA)) ||
        (s > 0 && (ldx < P->n || ldyl < P->n)))
        return rf_fail(P, RF_ERR_ARG, "bad arguments to rf_eig_vjp");
    const int64_t n = P->n;
    hipStream_t st = P->stream;
    if (s == 0) {
        if (P->A.nnz > 0) RF_HIP(P, hipMemsetAsync(gA, 0, sizeof(zd) * P->A.nnz, st));
        if (gB && P->B.nnz > 0) RF_HIP(P, hipMemsetAsync(gB, 0, sizeof(zd) * P->B.nnz, st));
        RF_HIP(P, hipStreamSynchronize(st));
        return RF_OK;
    }
    // pair every right eigenvalue with the adjoint eigenvalue whose conjugate is nearest
    const double scale = std::hypot(P->opts.c_re, P->opts.c_im) + P->opts.r;
    const double tol = 1e-6 * scale;
    std::vector<int> pair(s);
    std::vector<char> used(size_t(std::max(s_left, 1)), 0);
    for (int i = 0; i < s; ++i) {
        int best = -1;
        double bd = 0.0;
        for (int j = 0; j < s_left; ++j) {
            const double d = std::hypot(lambda[2 * i] - mu[2 * j], lambda[2 * i + 1] + mu[2 * j + 1]);
            if (best < 0 || d < bd) { best = j; bd = d; }
        }
        if (best < 0 || bd > tol || used[best])
            return rf_fail(P, RF_ERR_ARG, "eigenvalue " + std::to_string(i) +
                                              " has no unambiguous left partner in the adjoint results");
        used[best] = 1;
        pair[i] = best;
    }
    const zd *Xd = static_cast<const zd *>(X);
    const zd *Yd = static_cast<const zd *>(Yl);
    zd *dd = P->small;                 // s denominators
    zd *coef = P->small + s;           // s coefficients
    RF_HIP(P, hipMemcpyAsync(P->d_active, pair.data(), sizeof(int) * s, hipMemcpyHostToDevice, st));
    RF_HIP(P, launch_spmm(P->B, s, Xd, ldx, P->tmp, n, st));
    RF_HIP(P, launch_paired_dots(n, s, Yd, ldyl, P->d_active, P->tmp, n, dd, st));
    std::vector<zd> d(s), ca(s), cb(s);
    RF_HIP(P, hipMemcpyAsync(d.data(), dd, sizeof(zd) * s, hipMemcpyDeviceToHost, st));
    RF_HIP(P, hipStreamSynchronize(st));
    for (int i = 0; i < s; ++i) {
        const std::complex<double> di(d[i].x, d[i].y), gi(g[2 * i], g[2 * i + 1]),
            li(lambda[2 * i], lambda[2 * i + 1]);
        if (std::abs(di) == 0.0)
            return rf_fail(P, RF_ERR_ARG, "y^H B x = 0 for eigenvalue " + std::to_string(i) +
                                              " (not a simple eigenvalue)");
        const std::complex<double> a = gi / di, b = -gi * li / di;
        ca[i] = Z(a.real(), a.imag());
        cb[i] = Z(b.real(), b.imag());
        if (denom) { denom[2 * i] = d[i].x; denom[2 * i + 1] = d[i].y; }
        if (pair_out) pair_out[i] = pair[i];
    }
    RF_HIP(P, hipMemcpyAsync(coef, ca.data(), sizeof(zd) * s, hipMemcpyHostToDevice, st));
    RF_HIP(P, launch_sampled_outer(P->A, s, coef, Yd, ldyl, P->d_active, Xd, ldx,
                                   static_cast<zd *>(gA), st));
    RF_HIP(P, hipStreamSynchronize(st));
    if (gB) {
        RF_HIP(P, hipMemcpyAsync(coef, cb.data(), sizeof(zd) * s, hipMemcpyHostToDevice, st));
        RF_HIP(P, launch_sampled_outer(P->B, s, coef, Yd, ldyl, P->d_active, Xd, ldx,
                                       static_cast<zd *>(gB), st));
        RF_HIP(P, hipStreamSynchronize(st));
    }
    return RF_OK;
}

}  // extern "C"
