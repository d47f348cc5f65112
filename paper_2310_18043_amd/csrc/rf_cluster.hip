// Band solves of the inner rule G(X) = sum_i w_i K_i^{-1} B X by clusters of
// workgroups over fused factor tiles (Chen & Li, Sec. 3.2, eq. linearsolve2; the
// factors come from the pre-factorization loop of Alg. composite, rf_band.hip).
//
// The block-tridiagonal LU of K_i = p_i B - A gives, per block step k, the row order
// P_k of the 2nb-row window and the tiles Linv_k, L21_k, Uinv_k, U1_k, U2_k.  Formed
// once per factorization, the products
//     M_k = L21_k Linv_k,   W_k = Uinv_k Linv_k,   V1_k = Uinv_k U1_k,   V2_k = Uinv_k U2_k
// make each block step of the two sweeps depend on one whole intermediate block only:
//     forward,  w = P_k [t_k; b_{k+1}] (t_0 = b_0):   t_{k+1} = w_bot - M_k w_top,
//                                                     z_k     = W_k w_top
//     backward, x_nblk = x_{nblk+1} = 0:              x_k = z_k - V1_k x_{k+1} - V2_k x_{k+2}
// (z_k = U11^{-1} L11^{-1} w_top, so x_k is block row k of the back substitution).
//
// A cluster of C = nb / 16 workgroups owns one pole and 16 right-hand sides.  Member m
// computes rows 16m .. 16m+15 of every product on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; the four waves split the inner dimension and add their
// partial blocks in LDS), so a workgroup streams 1/C of its pole's tiles where the
// per-slice solve streams all of them for one or two columns.  The rows of t_{k+1} and
// x_k that a member produces reach the other members through an exchange area:
//   * the members of a cluster run on one XCD, so their stores and loads meet in that
//     XCD's L2: a workgroup reads its XCC id and takes a ticket from that XCD's counter
//     (reset before every launch), and cluster slot and member follow from (XCD,
//     ticket), in the order the workgroups arrive; a ticket past the XCD's share of the
//     grid is reported;
//   * a member stores its rows, waits until its stores are complete and then raises
//     its sequence flag, a 64-bit word (launch epoch << 32 | publication number);
//   * readers poll the flags and read the rows with agent-scope loads, which skip the
//     CU's L1 and so never see a stale line;
//   * two buffers alternate by the parity of the publication number: a member writes
//     publication s only after every member has raised s - 1, which each did only after
//     reading publication s - 2 from the buffer that s reuses.
// Every wait is bounded.  A member that gives up records the launch epoch in err[0];
// every later wait of the launch then returns at once and the host reports the error.
// Per step the product on the critical path (M_k forward, V1_k backward) is computed
// and published first; the other one (W_k, or V2_{k-1} x_{k+1} for the next step) runs
// while the flags propagate.  The tiles of the next step are loaded into registers
// while the current step runs.
//
// Cluster kernels of different streams could each hold part of the device while
// waiting for members that cannot start; the launcher therefore orders all cluster
// launches of a device one after another (an event chain), and a launch never has more
// workgroups than the device has compute units.
#include <mutex>
#include <type_traits>

#include "rf_common.h"

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));   // a complex tile entry in registers

constexpr int kClThreads = 256;
constexpr int kClRows = 16;          // rows of every product per member
constexpr int kClCols = 16;          // right-hand sides per cluster
constexpr int kRedLd = 17;           // padded row of a 16 x 16 partial block in LDS
constexpr int kVecLd = 17;           // padded row of the LDS vector block (16 columns)
constexpr int kFlagsPerSlot = 16;    // one 128-byte line of flags per cluster slot

struct ClusterArgs {
    int n, nblk, p, ncols;
    const zd *X;                        // right-hand sides B X: npad x ncols (ld npad), rows
                                        // n .. npad-1 zero
    const zd *ftiles;                   // [pole][k][4][nb x nb]: M, W, V1, V2 (column-major)
    const int32_t *perm;                // [pole][k][2nb]
    const zd *weights;                  // w_i
    const zd *colw;                     // or null: [pole][ncols] weights
    zd *zbuf;                           // [pole][npad x ncols]: z_k
    zd *xpart;                          // [pole][npad x ncols]: weighted solutions
    int64_t npad;
    int unit_weight, accumulate;
    zd *xchg;                           // [slot][2][C][16 x 16]
    unsigned long long *flags;          // [slot][16]
    unsigned *tickets;                  // [8 XCDs][32]: arrival counters, zero at launch
    unsigned *err;                      // [0] epoch of a timed-out wait, [1] of a misplaced member
    unsigned epoch;
    int nclusters, nslots;
    int spin_limit;
};

template <int NB>
struct ClShape {
    static constexpr int C = NB / kClRows;                            // members
    static constexpr int KW = NB / 4;                                 // inner range of a wave
    static constexpr int KS = KW / 4;                                 // MFMA steps per product
    static constexpr int GQ = (NB + kClRows) * kClCols / kClThreads;  // gathered entries per thread
    static constexpr int VEC = (NB + kClRows) * kVecLd;               // LDS vector + w_bot rows
    static constexpr int XQ = NB * kClCols / kClThreads;              // x entries per thread
    static constexpr int SLOT = kClRows * kClCols;                    // one member's block
    static constexpr int RED = kClRows * kRedLd;                      // one wave's partial block
    static_assert(C >= 2 && C <= kFlagsPerSlot && KS >= 1, "cluster shape");
    static_assert((NB + kClRows) * kClCols % kClThreads == 0, "gather shape");
};

template <int NB>
constexpr size_t cluster_lds() {
    return size_t(ClShape<NB>::VEC + 8 * ClShape<NB>::RED) * sizeof(zd);
}

__device__ __attribute__((always_inline)) inline dv4 mfma64(double a, double b, dv4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// This thread's A operands of one product: entry (row 16m + lane % 16, column
// wave KW + 4j + lane / 16) of the tile, for j = 0 .. KS-1 (t points at j = 0).
__device__ __attribute__((always_inline)) inline dv2 ld2(const zd *p) {
    return *reinterpret_cast<const dv2 *>(p);
}

template <int NB>
__device__ __attribute__((always_inline)) inline void cl_load(const zd *t,
                                                              dv2 (&buf)[ClShape<NB>::KS]) {
#pragma unroll
    for (int j = 0; j < ClShape<NB>::KS; ++j) buf[j] = ld2(t + int64_t(4 * j) * NB);
}

// red[wave] = this member's 16 rows of (tile x vec) over the wave's quarter of the inner
// dimension.  A (i, k) sits in lane i + 16k, B (k, j) in lane j + 16k, and the 16 x 16
// result entry (4r + lane / 16, lane % 16) in slot r; the four real products of the
// complex one accumulate separately.
// NL of the tiles pa, pb (0, 1 or 2) are loaded into da, db while the product runs: entry
// j of each right after the matrix-core instructions of step j, then ex(j), so that the
// loads' address work and issue overlap the matrix cores
struct ClNoExtra {
    __device__ void operator()(int) const {}
};

template <int NB, int NL, typename EX = ClNoExtra>
__device__ __attribute__((always_inline)) inline void cl_product(const dv2 (&t)[ClShape<NB>::KS],
                                                                 const zd *vec, zd *red, int wave,
                                                                 int lane, const zd *pa,
                                                                 dv2 (&da)[ClShape<NB>::KS],
                                                                 const zd *pb,
                                                                 dv2 (&db)[ClShape<NB>::KS],
                                                                 EX ex = EX()) {
    using S = ClShape<NB>;
    dv4 rr = {0.0, 0.0, 0.0, 0.0}, ii = rr, ri = rr, ir = rr;
    const zd *vb = vec + (wave * S::KW + (lane >> 4)) * kVecLd + (lane & 15);
#pragma unroll
    for (int j = 0; j < S::KS; ++j) {
        const zd b = vb[4 * j * kVecLd];
        rr = mfma64(t[j].x, b.x, rr);
        ii = mfma64(t[j].y, b.y, ii);
        ri = mfma64(t[j].x, b.y, ri);
        ir = mfma64(t[j].y, b.x, ir);
        if (NL >= 1) da[j] = ld2(pa + int64_t(4 * j) * NB);
        if (NL >= 2) db[j] = ld2(pb + int64_t(4 * j) * NB);
        ex(j);                                    // further loads of the caller
    }
    zd *dst = red + wave * S::RED + (lane >> 4) * kRedLd + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[4 * r * kRedLd] = zmake(rr[r] - ii[r], ri[r] + ir[r]);
}

// entry (lrow, col) of the product: the four waves' partial sums in fixed order
template <int NB>
__device__ __attribute__((always_inline)) inline zd cl_sum(const zd *red, int lrow, int col) {
    zd s = red[lrow * kRedLd + col];
#pragma unroll
    for (int w = 1; w < 4; ++w) s = zadd(s, red[w * ClShape<NB>::RED + lrow * kRedLd + col]);
    return s;
}

// Drop every line of this CU's L1 (vector) cache: after it, loads of this wave read the
// XCD's L2, where the other members' publications are.
__device__ __attribute__((always_inline)) inline void cl_inv_l1() {
    asm volatile("buffer_inv sc0" ::: "memory");
}

// The workgroup's stores are complete (in the XCD's L2) before its flag goes up.
__device__ __attribute__((always_inline)) inline void cl_raise(unsigned long long *flag,
                                                               unsigned long long v) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every member's flag has reached `target`, at most `limit` polls (the
// first wave polls, one lane per member).
template <int C>
__device__ inline void cl_wait(const unsigned long long *flags, unsigned long long target,
                               unsigned *err, unsigned epoch, int limit) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        unsigned long long *f = const_cast<unsigned long long *>(flags) + (lane < C ? lane : 0);
        for (int it = 0;; ++it) {
            const unsigned long long v = __hip_atomic_load(f, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            if (__all(lane >= C || v >= target)) break;
            if (it >= limit) {
                if (lane == 0)
                    __hip_atomic_store(err, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            if ((it & 63) == 63 &&
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch)
                break;
        }
    }
    __syncthreads();
}

// grid: nslots * C workgroups of 256 threads, nslots a multiple of 8, so each XCD runs
// nslots C / 8 of them: ticket t on XCD x makes a workgroup member t % C of slot
// (t / C) * 8 + x.  Slot s solves clusters s, s + nslots, ... (cluster c: pole c % p,
// right-hand sides 16 (c / p) ..).
template <int NB>
__global__ __launch_bounds__(kClThreads) void band_solve_cluster_kernel(ClusterArgs a) {
    using S = ClShape<NB>;
    constexpr int C = S::C, KW = S::KW, GQ = S::GQ, XQ = S::XQ, SLOT = S::SLOT;
    constexpr int64_t te = int64_t(NB) * NB;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const unsigned long long ep = (unsigned long long)a.epoch << 32;

    // 16-byte aligned: the static placement words below come first in LDS, and every
    // array here is read and written 16 bytes (one complex double) at a time
    extern __shared__ __align__(16) unsigned char smem_raw[];
    zd *vec = reinterpret_cast<zd *>(smem_raw);   // [NB][17]: w_top, later x_{k+1}
    zd *wbot = vec + NB * kVecLd;                 // [16][17]: this member's rows of w_bot
    zd *red0 = vec + S::VEC;                      // [4][16 x 17]: first product's partials
    zd *red1 = red0 + 4 * S::RED;                 // [4][16 x 17]: second product's partials

    __shared__ int s_place[2];
    if (tid == 0) {
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
        xcc &= 15u;
        int sl = -1, mm = 0;
        if (xcc < 8u) {
            const unsigned t = __hip_atomic_fetch_add(a.tickets + xcc * 32, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (t < unsigned(a.nslots / 8 * C)) {
                sl = int(t / C) * 8 + int(xcc);
                mm = int(t % C);
            }
        }
        if (sl < 0) __hip_atomic_store(a.err + 1, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_place[0] = sl;
        s_place[1] = mm;
    }
    __syncthreads();
    const int slot = __builtin_amdgcn_readfirstlane(s_place[0]);
    const int m = __builtin_amdgcn_readfirstlane(s_place[1]);
    // a workgroup past its XCD's share leaves; the members that would wait for it give up
    // after the bounded wait, and the launch is reported
    if (slot < 0) return;

    const int lrow = tid & 15, oc = tid >> 4;     // this thread's entry of a 16 x 16 block
    unsigned long long *myflag = a.flags + int64_t(slot) * kFlagsPerSlot + m;
    const unsigned long long *cflags = a.flags + int64_t(slot) * kFlagsPerSlot;
    zd *xch = a.xchg + int64_t(slot) * 2 * C * SLOT;
    unsigned seq = 0;                             // publications of this launch so far
    const int nblk = a.nblk;

    for (int cl = slot; cl < a.nclusters; cl += a.nslots) {
        const int pole = cl % a.p, c0 = (cl / a.p) * kClCols;
        const zd *F = a.ftiles + int64_t(pole) * nblk * 4 * te + 16 * m + (lane & 15) +
                      int64_t(wave * KW + (lane >> 4)) * NB;
        auto tile = [&](int k, int t) __attribute__((always_inline)) {
            return F + (int64_t(k) * 4 + t) * te;
        };
        const int32_t *perm = a.perm + int64_t(pole) * nblk * 2 * NB;
        zd *zb = a.zbuf + int64_t(pole) * a.npad * a.ncols;
        zd *xp = a.xpart + int64_t(pole) * a.npad * a.ncols;
        const int col = c0 + oc;
        const bool colok = col < a.ncols;
        const int64_t zoff = 16 * m + lrow + int64_t(colok ? col : 0) * a.npad;

        // entry (row, column cc of the cluster) of B X, row < npad.  Columns past ncols
        // read the last column: each right-hand side is solved on its own, so those lanes
        // only produce outputs that are not stored.
        auto rhs = [&](int64_t row, int cc) __attribute__((always_inline)) -> dv2 {
            const int cg = min(c0 + cc, a.ncols - 1);
            return ld2(a.X + row + int64_t(cg) * a.npad);
        };
        auto zload = [&](int k) __attribute__((always_inline)) -> zd {
            return (k >= 0 && colok) ? zb[int64_t(k) * NB + zoff] : zmake(0.0, 0.0);
        };
        // this thread's weight: w_i, the per-column weight, or 1
        const zd wc = a.unit_weight ? zmake(1.0, 0.0)
                    : a.colw ? a.colw[int64_t(pole) * a.ncols + (colok ? col : 0)] : a.weights[pole];
        auto out = [&](int k, zd v) __attribute__((always_inline)) {
            if (!colok) return;
            zd *dst = xp + int64_t(k) * NB + zoff;
            const zd val = zmul(wc, v);
            if (a.accumulate) *dst = zadd(*dst, val);
            else *dst = val;
        };

        // gathered entry q of w_k (rows(k) window rows: NB + 16 while a block follows,
        // else NB): e = tid + 256 q, window row i = e % rows(k) (i < NB: w_top row i; else
        // this member's w_bot row i - NB), column e / rows(k).  Consecutive lanes take
        // consecutive rows of one column, which are adjacent in X and in the exchange area.
        // window rows of w_k (the permutation), B X entries and t_k entries per thread
        int pa_[GQ], pb_[GQ];
        dv2 gv[GQ], gt[GQ];
        // the two window heights as compile-time constants (cheap divisions by rows)
        using Full = std::integral_constant<int, NB + kClRows>;
        using Last = std::integral_constant<int, NB>;
        // full windows (a block follows): per entry q the window row index into the
        // permutation and the B X column, fixed for the whole sweep
        int fpi[GQ];
        const zd *fxc[GQ];
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
            constexpr int rows = NB + kClRows;
            const int e = tid + q * kClThreads, i = e % rows, cc = e / rows;
            fpi[q] = i < NB ? i : NB + 16 * m + (i - NB);
            fxc[q] = a.X + int64_t(min(c0 + cc, a.ncols - 1)) * a.npad;
        }
        // entry q of the permutation of block k, as stored (read where it is used through
        // wrow, which keeps it to the window's rows, so no loaded value is tested here)
        auto perm_q_r = [&](auto R_, int k, int q, int (&ps)[GQ]) __attribute__((always_inline)) {
            constexpr int rows = decltype(R_)::value;
            const int e = tid + q * kClThreads, i = e % rows;
            const int pi = i < NB ? i : NB + 16 * m + (i - NB);
            if (e < rows * kClCols) ps[q] = perm[int64_t(k) * 2 * NB + pi];
        };
        auto wrow = [](int v) __attribute__((always_inline)) { return min(max(v, 0), 2 * NB - 1); };
        // entry q of w_k as if it came from b: window row src is row k NB + src of B X
        // (block k for src < NB, block k+1 after); for k > 0 the entries with src < NB are
        // replaced by rows of t_k.  While block k+1 exists no loaded value is tested, so
        // the loads are only waited for where the window is stored.
        auto gather_b_r = [&](auto R_, int k, int q, const int (&ps)[GQ]) __attribute__((always_inline)) {
            constexpr int rows = decltype(R_)::value;
            const int e = tid + q * kClThreads, cc = e / rows;
            if (e >= rows * kClCols) return;
            const int src = wrow(ps[q]);
            const int64_t row = int64_t(k) * NB + src;
            if (k + 2 <= nblk) gv[q] = rhs(row, cc);
            else gv[q] = src < NB ? rhs(row, cc) : dv2{0.0, 0.0};    // last block: no b_{k+1}
        };
        // all entries of w_k that come from b; one branch around straight-line loads (a
        // branch per entry would make the loads wait for each other)
        auto gather_b = [&](int k, const int (&ps)[GQ]) __attribute__((always_inline)) {
            if (k + 1 < nblk) {                                    // block k+1 exists
#pragma unroll
                for (int q = 0; q < GQ; ++q) gv[q] = ld2(fxc[q] + int64_t(k) * NB + wrow(ps[q]));
            } else {
#pragma unroll
                for (int q = 0; q < GQ; ++q) gather_b_r(Last(), k, q, ps);
            }
        };
        auto load_perm = [&](int k, int (&ps)[GQ]) __attribute__((always_inline)) {
            if (k + 1 < nblk) {
#pragma unroll
                for (int q = 0; q < GQ; ++q) ps[q] = perm[int64_t(k) * 2 * NB + fpi[q]];
            } else {
#pragma unroll
                for (int q = 0; q < GQ; ++q) perm_q_r(Last(), k, q, ps);
            }
        };
        // the published rows of t_k at the window rows, loaded for every entry (rows of b
        // read a harmless row of t) and chosen where the window is stored
        auto gather_t_r = [&](auto R_, const zd *pub, const int (&ps)[GQ]) __attribute__((always_inline)) {
            constexpr int rows = decltype(R_)::value;
#pragma unroll
            for (int q = 0; q < GQ; ++q) {
                const int e = tid + q * kClThreads, cc = e / rows;
                const int src = wrow(ps[q]) & (NB - 1);
                if (e < rows * kClCols) gt[q] = ld2(pub + (src >> 4) * SLOT + cc * 16 + (src & 15));
            }
        };
        auto store_w_r = [&](auto R_, bool with_t, const int (&ps)[GQ]) __attribute__((always_inline)) {
            constexpr int rows = decltype(R_)::value;
#pragma unroll
            for (int q = 0; q < GQ; ++q) {
                const int e = tid + q * kClThreads, i = e % rows, cc = e / rows;
                if (e >= rows * kClCols) continue;
                const dv2 v = (with_t && wrow(ps[q]) < NB) ? gt[q] : gv[q];
                vec[i * kVecLd + cc] = zmake(v.x, v.y);   // rows NB.. : w_bot
            }
        };
        auto gather_t = [&](int k, const zd *pub, const int (&ps)[GQ]) __attribute__((always_inline)) {
            cl_inv_l1();
            if (k + 1 < nblk) gather_t_r(Full(), pub, ps); else gather_t_r(Last(), pub, ps);
        };
        auto store_w = [&](int k, bool with_t, const int (&ps)[GQ]) __attribute__((always_inline)) {
            if (k + 1 < nblk) store_w_r(Full(), with_t, ps); else store_w_r(Last(), with_t, ps);
        };
        auto load_x = [&](const zd *pub) __attribute__((always_inline)) {
            cl_inv_l1();
            dv2 xv[XQ];
#pragma unroll
            for (int q = 0; q < XQ; ++q) {
                const int e = tid + q * kClThreads, i = e % NB, cc = e / NB;
                xv[q] = ld2(pub + (i >> 4) * SLOT + cc * 16 + (i & 15));
            }
#pragma unroll
            for (int q = 0; q < XQ; ++q) {
                const int e = tid + q * kClThreads, i = e % NB, cc = e / NB;
                vec[i * kVecLd + cc] = zmake(xv[q].x, xv[q].y);
            }
        };
        auto publish = [&](zd v) __attribute__((always_inline)) {
            ++seq;
            xch[(seq & 1) * C * SLOT + m * SLOT + oc * 16 + lrow] = v;
            cl_raise(myflag, ep | seq);
        };
        auto wait_all = [&]() __attribute__((always_inline)) {
            cl_wait<C>(cflags, ep | seq, a.err, a.epoch, a.spin_limit);
        };
        const zd *const pub0 = xch;                   // buffer of even publications
        auto pub = [&]() __attribute__((always_inline)) { return pub0 + (seq & 1) * C * SLOT; };

        // ---------------- forward sweep
        // Tiles: ta holds the first product of the coming step (M_k, later V1_k); the
        // second product's tile alternates between tb and tc, so that all loads of step
        // k+1 are issued right after the publication of step k (whose wait for completed
        // stores then finds the previous step's loads long done).  The loops are unrolled
        // by two so that every buffer is a fixed register set.
        dv2 ta[S::KS], tb[S::KS], tc[S::KS];
        load_perm(0, pa_);
        gather_b(0, pa_);
        store_w(0, false, pa_);
        if (nblk > 1) cl_load<NB>(tile(0, 0), ta);    // M_0
        cl_load<NB>(tile(0, 1), tb);                  // W_0
        if (nblk > 1) load_perm(1, pb_);
        __syncthreads();
        zd pre = zmake(0.0, 0.0), zcur = zmake(0.0, 0.0);

        // forward step k < nblk - 1, second tile in tcur, the next one into tnext
        // pcur holds the permutation of block k+1; that of block k+2 goes into pnext
        auto fwd = [&](int k, dv2 (&tcur)[S::KS], dv2 (&tnext)[S::KS], int (&pcur)[GQ],
                       int (&pnext)[GQ]) __attribute__((always_inline)) {
            // t_{k+1} = w_bot - M_k w_top
            cl_product<NB, 0>(ta, vec, red0, wave, lane, nullptr, ta, nullptr, ta);
            __syncthreads();
            publish(zsub(wbot[lrow * kVecLd + oc], cl_sum<NB>(red0, lrow, oc)));
            // the rows of w_{k+1} that come from b and the permutation of block k+2 are
            // requested first (ahead of the tile stream in the CU's queue); then
            // z_k = W_k w_top while M_{k+1} (or V1_{nblk-2}) and W_{k+1} are requested
            gather_b(k + 1, pcur);
            if (k + 2 < nblk) load_perm(k + 2, pnext);
            const zd *na = k + 2 < nblk ? tile(k + 1, 0) : tile(nblk - 2, 2);
            const zd *nw = tile(k + 1, 1);
            cl_product<NB, 2>(tcur, vec, red1, wave, lane, na, ta, nw, tnext);
            __syncthreads();
            const zd zv = cl_sum<NB>(red1, lrow, oc);
            if (colok) zb[int64_t(k) * NB + zoff] = zv;
            wait_all();
            gather_t(k + 1, pub(), pcur);                                // w_{k+1}: rows of t
            store_w(k + 1, true, pcur);
            __syncthreads();
        };
        // backward step k >= 1: ta = V1_k, tcur = V2_{k-1}, the next V2 into tnext
        auto bwd = [&](int k, dv2 (&tcur)[S::KS], dv2 (&tnext)[S::KS]) __attribute__((always_inline)) {
            cl_product<NB, 0>(ta, vec, red0, wave, lane, nullptr, ta, nullptr, ta);
            __syncthreads();
            const zd xv = zsub(pre, cl_sum<NB>(red0, lrow, oc));
            publish(xv);
            const zd znext = zload(k - 2);
            out(k, xv);
            // V2_{k-1} x_{k+1}, while V1_{k-1} and V2_{k-2} are requested (at k = 1 the
            // second load reads V2_0 again, unused: one code path for every step)
            const zd *na = tile(k - 1, 2);
            const zd *nv = tile(k >= 2 ? k - 2 : 0, 3);
            cl_product<NB, 2>(tcur, vec, red1, wave, lane, na, ta, nv, tnext);
            __syncthreads();
            pre = zsub(zcur, cl_sum<NB>(red1, lrow, oc));
            zcur = znext;
            wait_all();
            load_x(pub());
            __syncthreads();
        };
        // last block, then the backward sweep; W_{nblk-1} in t0
        auto finish = [&](dv2 (&t0)[S::KS], dv2 (&t1)[S::KS]) __attribute__((always_inline)) {
            // x_{nblk-1} = z_{nblk-1}
            cl_product<NB, 0>(t0, vec, red1, wave, lane, nullptr, t0, nullptr, t0);
            __syncthreads();
            const zd zv = cl_sum<NB>(red1, lrow, oc);
            if (nblk < 2) {
                out(0, zv);
                return;
            }
            publish(zv);
            if (nblk >= 3) cl_load<NB>(tile(nblk - 3, 3), t1);          // V2_{nblk-3}
            out(nblk - 1, zv);
            pre = zload(nblk - 2);                                       // pre_{nblk-2} = z_{nblk-2}
            zcur = zload(nblk - 3);
            wait_all();
            load_x(pub());
            __syncthreads();
            // vec = x_{k+1}, pre = z_k - V2_k x_{k+2}, zcur = z_{k-1}, ta = V1_k
            int k = nblk - 2;
            for (; k >= 2; k -= 2) {
                bwd(k, t1, t0);
                bwd(k - 1, t0, t1);
            }
            if (k == 1) bwd(1, t1, t0);
            cl_product<NB, 0>(ta, vec, red0, wave, lane, nullptr, ta, nullptr, ta);   // x_0
            __syncthreads();
            out(0, zsub(pre, cl_sum<NB>(red0, lrow, oc)));
        };
        int k = 0;
        for (; k + 2 < nblk; k += 2) {
            fwd(k, tb, tc, pb_, pa_);
            fwd(k + 1, tc, tb, pa_, pb_);
        }
        if (k + 1 < nblk) {
            fwd(k, tb, tc, pb_, pa_);
#pragma unroll
            for (int j = 0; j < S::KS; ++j) tb[j] = tc[j];   // W_{nblk-1} into tb (registers)
        }
        finish(tb, tc);
        __syncthreads();                              // LDS is reused by the next cluster
    }
}

// Y (row, col) = d[row] X (row, col) for rows < n (d null: 1), 0 for rows n .. npad-1;
// Y is npad x ncols (ld npad) and may be X itself (then ldx = npad)
__global__ void stage_kernel(int64_t n, int64_t npad, int ncols, const zd *d, const zd *X,
                             int64_t ldx, zd *Y, unsigned *tickets) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < 8) tickets[e * 32] = 0u;          // the cluster kernel's arrival counters
    if (e >= npad * ncols) return;
    const int64_t r = e % npad, c = e / npad;
    zd v = zmake(0.0, 0.0);
    if (r < n) {
        v = X[r + c * ldx];
        if (d) v = zmul(d[r], v);
    }
    Y[r + c * npad] = v;
}

// Fused tiles of one product type for every (pole, block): C_t = A_t B_t.
hipError_t fused_product(const rf_plan &P, int a_slot, int b_slot, int c_slot, hipStream_t s) {
    const int nb = P.F.nb;
    const int64_t te = P.F.tile_elems;
    const int batch = P.opts.p * P.F.nblk;
    return launch_gemm_nn(nb, nb, nb, zmake(1.0, 0.0), P.F.tiles + a_slot * te, nb, 5 * te,
                          P.F.tiles + b_slot * te, nb, 5 * te, zmake(0.0, 0.0),
                          P.F.ftiles + c_slot * te, nb, 4 * te, batch, s);
}

// Per device: the event that the last cluster launch recorded (launch order).
constexpr int kMaxDev = 64;
struct ClusterGate {
    std::mutex mu;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int last = -1;
    bool ready = false;
};
ClusterGate g_gate[kMaxDev];

template <int NB>
hipError_t launch_nb(const ClusterArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(band_solve_cluster_kernel<NB>, dim3(grid), dim3(kClThreads),
                       cluster_lds<NB>(), s, a);
    return hipGetLastError();
}

}  // namespace

// tiles 64 and 128 (at 256 the kernel's registers do not hold a step's tiles: the
// per-slice solve runs there)
bool cluster_solve_supported(int nb) { return nb == 64 || nb == 128; }

int cluster_slots_max(int nb, int num_cu) {
    const int C = nb / kClRows;
    const int per = (num_cu / C) / 8 * 8;
    return per < 8 ? 8 : per;
}

size_t cluster_xchg_elems(int nb, int num_cu) {
    return size_t(cluster_slots_max(nb, num_cu)) * 2 * (nb / kClRows) * kClRows * kClCols;
}

size_t cluster_flag_words(int nb, int num_cu) {
    return size_t(cluster_slots_max(nb, num_cu)) * kFlagsPerSlot;
}

hipError_t cluster_gate_init(int device) {
    if (device < 0 || device >= kMaxDev) return hipErrorInvalidDevice;
    ClusterGate &g = g_gate[device];
    std::lock_guard<std::mutex> lock(g.mu);
    if (g.ready) return hipSuccess;
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipEventCreateWithFlags(&g.ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    g.ready = true;
    return hipSuccess;
}

hipError_t launch_fused_tiles(const rf_plan &P, hipStream_t s) {
    if (!P.F.ftiles || !P.F.tiles) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = fused_product(P, 1, 0, 0, s)) != hipSuccess) return e;   // M  = L21 Linv
    if ((e = fused_product(P, 2, 0, 1, s)) != hipSuccess) return e;   // W  = Uinv Linv
    if ((e = fused_product(P, 2, 3, 2, s)) != hipSuccess) return e;   // V1 = Uinv U1
    return fused_product(P, 2, 4, 3, s);                               // V2 = Uinv U2
}

hipError_t launch_cluster_solve(const rf_plan &P, const ClusterSolve &cs, hipStream_t s) {
    const int nb = P.F.nb;
    if (!cluster_solve_supported(nb) || !P.F.ftiles || !P.F.xchg || !P.F.cflags || !P.F.cerr ||
        !P.F.ctickets)
        return hipErrorInvalidValue;
    if (P.device < 0 || P.device >= kMaxDev || !g_gate[P.device].ready) return hipErrorNotReady;
    const int C = nb / kClRows;
    ClusterArgs a;
    a.n = int(P.n); a.nblk = P.F.nblk; a.p = P.opts.p; a.ncols = cs.ncols;
    a.npad = int64_t(P.F.nblk) * nb;
    // B X staged as npad x ncols with zero rows past n (in place when X is the stage)
    if (!cs.stage || cs.x_pole_stride != 0) return hipErrorInvalidValue;
    {
        const int64_t tot = a.npad * int64_t(cs.ncols);
        hipLaunchKernelGGL(stage_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, P.n,
                           a.npad, cs.ncols, cs.bdiag, cs.X, cs.ldx, cs.stage, P.F.ctickets);
        hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return e0;
        a.X = cs.stage;
    }
    a.ftiles = P.F.ftiles; a.perm = P.F.perm;
    a.weights = P.d_weights; a.colw = cs.colw;
    a.zbuf = cs.zbuf; a.xpart = cs.xpart;
    a.unit_weight = cs.unit_weight; a.accumulate = cs.accumulate;
    a.xchg = P.F.xchg; a.flags = P.F.cflags; a.err = P.F.cerr; a.tickets = P.F.ctickets;
    a.epoch = ++P.F.cepoch;
    a.nclusters = a.p * ((cs.ncols + kClCols - 1) / kClCols);
    const int smax = cluster_slots_max(nb, P.num_cu);
    a.nslots = std::min(smax, (a.nclusters + 7) / 8 * 8);
    a.spin_limit = 1 << 22;
    const int grid = a.nslots * C;
    if (a.nclusters <= 0) return hipSuccess;

    ClusterGate &g = g_gate[P.device];
    std::lock_guard<std::mutex> lock(g.mu);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return e;
    const bool chain = cap == hipStreamCaptureStatusNone;
    if (chain && g.last >= 0 && (e = hipStreamWaitEvent(s, g.ev[g.last], 0)) != hipSuccess) return e;
    e = nb == 64 ? launch_nb<64>(a, grid, s) : launch_nb<128>(a, grid, s);
    if (e != hipSuccess) return e;
    if (chain) {
        const int next = g.last == 0 ? 1 : 0;
        if ((e = hipEventRecord(g.ev[next], s)) != hipSuccess) return e;
        g.last = next;
    }
    return hipSuccess;
}
