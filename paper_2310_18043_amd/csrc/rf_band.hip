// Band LU of the shifted pencils K_i = p_i B - A and the multi-RHS solves of the
// inner rule G(X) = sum_i w_i K_i^{-1} B X  (Chen & Li, Sec. 3.2, eq. linearsolve2,
// the pre-factorization loop of Alg. composite).
//
// Block-tridiagonal form.  With a tile size nb >= max(kl, ku) the band matrix is
// block tridiagonal in nb x nb tiles.  LU with partial pivoting keeps that shape:
// at block step k the pivot search for the panel (column block k) only sees the
// 2nb rows of row blocks k and k+1, and the U block row k reaches column blocks
// k, k+1 and k+2.  Per pole and per block step k the factorization stores
//   perm_k : the row permutation of the 2nb-row window [row block k; row block k+1]
//   Linv_k : inverse of the unit lower triangle L11 of the panel
//   L21_k  : the multipliers of row block k+1
//   Uinv_k : inverse of the upper triangle U11
//   U1_k, U2_k : U block row k in column blocks k+1, k+2
// so that the forward sweep is, per step,  w = P_k [t_k; b_{k+1}],
// y_k = Linv_k w_top,  t_{k+1} = w_bot - L21_k y_k,  and the backward sweep is
// x_k = Uinv_k (y_k - U1_k x_{k+1} - U2_k x_{k+2}).  Every step of both sweeps
// is a pair or triple of dense nb x nb times nb x cols products, so the solve is
// a stream of coalesced tile reads.  Inverting the two diagonal triangles once
// at factorization time turns the triangular solves into the same products.
//
// Rows beyond n are padded with the identity so that every block is full.
#include <mutex>

#include "rf_common.h"

namespace {

constexpr int kThreads = 256;

struct FactorArgs {
    int n;              // true size
    int nb, nblk;
    // CSR of A and B (device)
    const int32_t *arow, *acol; const zd *aval;
    const int32_t *brow, *bcol; const zd *bval;
    const zd *poles;
    zd *tiles;          // [pole][k][5][nb*nb]
    int32_t *perm;      // [pole][k][2nb]
    zd *window;         // [pole][2][2nb x 3nb], ld 2nb (double-buffered)
    zd *rows;           // [pole][nblk][nb x 3nb], ld nb: prepared row blocks
    int32_t *subperm;   // [pole][2nb]: row order of the current sub-panel
    int32_t *info;      // [pole]
};

__device__ inline int64_t tile_index(int pole, int k, int t, int nblk, int64_t te) {
    return ((int64_t(pole) * nblk + k) * 5 + t) * te;
}

// Scatter row block `rb` of K = z B - A into window rows [h*nb, h*nb+nb),
// with window column 0 = global column `cbase`.  Rows >= n get the identity.
__device__ void scatter_rows(const FactorArgs &a, zd z, zd *W, int ldw, int h, int rb,
                             int cbase) {
    const int nb = a.nb;
    for (int ii = threadIdx.x; ii < nb; ii += blockDim.x) {
        int i = rb * nb + ii;
        int wr = h * nb + ii;
        if (i >= a.n) {
            int wc = i - cbase;
            if (wc >= 0 && wc < 3 * nb) W[wr + int64_t(wc) * ldw] = zmake(1.0, 0.0);
            continue;
        }
        for (int e = a.arow[i]; e < a.arow[i + 1]; ++e) {
            int wc = a.acol[e] - cbase;
            if (wc >= 0 && wc < 3 * nb) {
                zd v = W[wr + int64_t(wc) * ldw];
                W[wr + int64_t(wc) * ldw] = zsub(v, a.aval[e]);
            }
        }
        for (int e = a.brow[i]; e < a.brow[i + 1]; ++e) {
            int wc = a.bcol[e] - cbase;
            if (wc >= 0 && wc < 3 * nb) {
                zd v = W[wr + int64_t(wc) * ldw];
                zfma(v, z, a.bval[e]);
                W[wr + int64_t(wc) * ldw] = v;
            }
        }
    }
}

__device__ inline zd *pole_window(zd *base, int pole, int buf, int nb) {
    return base + (int64_t(pole) * 2 + buf) * (2 * nb) * (3 * nb);
}

// Row block rb of K = z B - A for every pole, prepared once per factorization:
// nb x 3nb, column-major (ld nb), column 0 = global column (rb - 1) nb.
// grid: (nblk, p)
__global__ __launch_bounds__(256) void rowblock_prep_kernel(FactorArgs a) {
    const int rb = blockIdx.x, pole = blockIdx.y;
    const int nb = a.nb;
    const int64_t tot = int64_t(nb) * 3 * nb;
    zd *Pb = a.rows + (int64_t(pole) * a.nblk + rb) * tot;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) Pb[e] = zmake(0, 0);
    __syncthreads();
    scatter_rows(a, a.poles[pole], Pb, nb, 0, rb, (rb - 1) * nb);
}

// First window of every pole: row blocks 0 and 1, window column 0 = global column 0.
__global__ __launch_bounds__(256) void band_window_init_kernel(FactorArgs a) {
    const int pole = blockIdx.x;
    const int nb = a.nb, ldw = 2 * nb;
    zd *W = pole_window(a.window, pole, 0, nb);
    const int64_t tot = int64_t(nb) * 3 * nb;
    const zd *P0 = a.rows + int64_t(pole) * a.nblk * tot;
    const zd *P1 = P0 + tot;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
        int r = int(e % nb), c = int(e / nb);
        // row block 0 is stored from global column -nb
        W[r + int64_t(c) * ldw] = (c < 2 * nb) ? P0[r + int64_t(c + nb) * nb] : zmake(0, 0);
        W[nb + r + int64_t(c) * ldw] = (a.nblk > 1) ? P1[e] : zmake(0, 0);
    }
    if (threadIdx.x == 0) a.info[pole] = 0;
}

// The factorization of block step k runs as nb/SW sub-steps of SW columns
// (right-looking, blocked), each one pair of launches for all p poles:
//   band_panel_kernel (one workgroup per pole): LU with partial pivoting of the
//       R x SW sub-panel (window columns c0..c0+SW-1) held in registers, one
//       window row per thread, one barrier per column.  Writes the sub-panel back,
//       its row permutation (subperm) and the running permutation of the block step.
//   band_trail_kernel (one wave per window column, many workgroups per pole):
//       columns right of the sub-panel: gather in the sub-panel's row order, solve
//       with its unit lower SW x SW block, subtract L * U from the rows below;
//       columns left of it: apply the permutation.  The last sub-step writes the
//       tiles (packed L11\U11, L21, U1, U2), the top half of the next window, and
//       copies the prepared row block k+2 into its bottom half.
// Kernel boundaries order the sub-steps, so no workgroup ever waits on another.
constexpr int kFacThreads = 512;
constexpr int kFacWaves = kFacThreads / 64;

// Wave-wide maximum of a 64-bit key with DPP moves: within each row of 16 lanes by
// shifts of 1, 2, 4, 8, then across rows by the row-15 and row-31 broadcasts; lane
// 63 ends with the maximum.  Lanes whose DPP source does not exist keep their own
// value.  A non-negative double's bit pattern orders like the double, so the keys
// are the bits of |a|^2.
__device__ __attribute__((always_inline)) inline uint64_t wave_max_u64(uint64_t key) {
#define RF_MAX_STEP(CTRL, ROWMASK)                                                            \
    {                                                                                         \
        const int lo = int(uint32_t(key)), hi = int(uint32_t(key >> 32));                     \
        const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);       \
        const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);       \
        const uint64_t o = (uint64_t(uint32_t(ohi)) << 32) | uint32_t(olo);                   \
        key = o > key ? o : key;                                                              \
    }
    RF_MAX_STEP(0x111, 0xF)     // row_shr:1
    RF_MAX_STEP(0x112, 0xF)     // row_shr:2
    RF_MAX_STEP(0x114, 0xF)     // row_shr:4
    RF_MAX_STEP(0x118, 0xF)     // row_shr:8
    RF_MAX_STEP(0x142, 0xA)     // row_bcast:15 into rows 1 and 3
    RF_MAX_STEP(0x143, 0xC)     // row_bcast:31 into rows 2 and 3
#undef RF_MAX_STEP
    return key;
}

struct PivotCand {
    uint64_t key;       // bits of |a|^2 (0: no candidate or exact zero)
    int tid;            // thread holding the row
    int pos;            // its current position in the window
};

// One workgroup per pole, one thread per window row (row `tid` of the window at the
// start of the sub-step, R live rows), the row's SW sub-panel entries in registers.
// Partial pivoting by largest |.|^2 over the rows at positions >= the current
// column (ties: lowest thread).  Interchanges are not carried out: every thread keeps
// the position of its row, and the pivot row and the row at the pivot position trade
// positions, so row interchanges of the whole sub-panel (the multipliers of earlier
// columns included) come for free.  Per column: the candidate of each wave (DPP max,
// ballot) writes a record (key, thread, position) to LDS, one barrier, every thread
// picks the winner among the waves' records, the winning thread stores its row from the
// pivot column on, a second barrier, and every thread updates its own row.  (Every wave
// storing its candidate's row before a single barrier costs more: a wave's LDS stores
// issue one at a time, some tens of cycles each, so four waves' rows took longer than
// one row and a barrier.)  The rows are written back at their new positions, with the
// sub-panel's row order (subperm) and the running permutation of the block step.
template <int SW, int NT>
__global__ __launch_bounds__(NT) void band_panel_kernel(FactorArgs a, int k, int buf, int c0) {
    constexpr int NWMAX = NT / 64;
    const int pole = blockIdx.x;
    const int nb = a.nb, nblk = a.nblk, ldw = 2 * nb;
    zd *W = pole_window(a.window, pole, buf, nb);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nw = int(blockDim.x) >> 6;
    const int R = (k + 1 < nblk) ? 2 * nb : nb;
    const bool live = tid < R;
    __shared__ PivotCand cand[NWMAX];
    __shared__ zd urow[SW];
    __shared__ int s_pm[NT];
    int32_t *pm = a.perm + (int64_t(pole) * nblk + k) * (2 * nb);
    // the running permutation is read before the first barrier and written after the
    // last one (through LDS, so that every read has landed before any thread writes)
    if (tid < 2 * nb) s_pm[tid] = (c0 == 0) ? tid : pm[tid];
    zd x[SW];
#pragma unroll
    for (int j = 0; j < SW; ++j) x[j] = live ? W[tid + int64_t(c0 + j) * ldw] : zmake(0, 0);
    // the pivot row starts finite (a singular column reads it, times zero)
    if (tid < SW) urow[tid] = zmake(0, 0);
    // waves that do not exist never offer a candidate
    if (tid < NWMAX && tid >= nw) {
        cand[tid].key = 0;
        cand[tid].tid = -1;
        cand[tid].pos = -1;
    }
    // the initialisation above must land before the first candidates are written
    __syncthreads();
    int pos = tid;
    int info = 0;
#pragma unroll
    for (int j = 0; j < SW; ++j) {
        const int gj = c0 + j;
        const bool is_cand = live && pos >= gj;
        const double m = zabs2(x[j]);
        const uint64_t mine = (is_cand && m > 0.0) ? uint64_t(__double_as_longlong(m)) : 0;
        const uint64_t top = wave_max_u64(mine);
        const uint64_t wmax =
            (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(top >> 32)), 63))) << 32) |
            uint32_t(__builtin_amdgcn_readlane(int(uint32_t(top)), 63));
        const uint64_t hit = __ballot(is_cand && mine == wmax);
        if (hit != 0 && lane == int(__builtin_ctzll(hit))) {
            PivotCand c;
            c.key = wmax; c.tid = tid; c.pos = pos;
            cand[wave] = c;
        } else if (hit == 0 && lane == 0) {
            PivotCand c;
            c.key = 0; c.tid = -1; c.pos = -1;
            cand[wave] = c;
        }
        __syncthreads();
        // winner: largest nonzero key, ties to the lowest wave (so the lowest thread);
        // none: singular column (no interchange, zero multipliers)
        PivotCand cw[NWMAX];
#pragma unroll
        for (int w = 0; w < NWMAX; ++w) cw[w] = cand[w];
        uint64_t bk = 0;
        int tw = -1, pw = gj;
#pragma unroll
        for (int w = 0; w < NWMAX; ++w)
            if (cw[w].key > bk) { bk = cw[w].key; tw = cw[w].tid; pw = cw[w].pos; }
        tw = __builtin_amdgcn_readfirstlane(tw);
        pw = __builtin_amdgcn_readfirstlane(pw);
        const bool sing = tw < 0;
        if (sing && info == 0) info = k * nb + gj + 1;
        // only the winning row goes through LDS (a wave's LDS stores issue one at a time)
        if (tid == tw) {
#pragma unroll
            for (int q = j; q < SW; ++q) urow[q] = x[q];
        }
        __syncthreads();
        const zd *ur = urow;
        const zd uj = ur[j];
        // 1 / u_j = conj(u_j) / |u_j|^2 (the pivot is the column's largest entry)
        const double sc = 1.0 / zabs2(uj);
        pos = (tid == tw) ? gj : (pos == gj ? pw : pos);
        const bool upd = live && pos > gj;
        const zd xl = zmake(x[j].x * uj.x + x[j].y * uj.y, x[j].y * uj.x - x[j].x * uj.y);
        const zd l = (upd && !sing) ? zmake(xl.x * sc, xl.y * sc) : zmake(0, 0);
        if (upd) x[j] = l;
#pragma unroll
        for (int q = j + 1; q < SW; ++q) zfms(x[q], l, ur[q]);
    }
    if (live && pos >= c0) {
#pragma unroll
        for (int j = 0; j < SW; ++j) W[pos + int64_t(c0 + j) * ldw] = x[j];
    }
    int32_t *sp = a.subperm + int64_t(pole) * 2 * nb;
    if (tid < 2 * nb) {
        sp[pos] = tid;
        pm[pos] = s_pm[tid];
    }
    if (tid == 0 && info != 0 && a.info[pole] == 0) a.info[pole] = info;
}

// value of x in lane ln (ln wave-uniform): four readlanes, no LDS round trip
__device__ __attribute__((always_inline)) inline zd lane_bcast(zd x, int ln) {
    const int a = __builtin_amdgcn_readlane(__double2loint(x.x), ln);
    const int b = __builtin_amdgcn_readlane(__double2hiint(x.x), ln);
    const int c = __builtin_amdgcn_readlane(__double2loint(x.y), ln);
    const int d = __builtin_amdgcn_readlane(__double2hiint(x.y), ln);
    return zmake(__hiloint2double(b, a), __hiloint2double(d, c));
}

// grid: (ceil(columns / 8), p); one window column per wave.
template <int NS, int SW>
__global__ __launch_bounds__(kFacThreads) void band_trail_kernel(FactorArgs a, int k, int buf,
                                                                int c0) {
    const int pole = blockIdx.y;
    const int nb = a.nb, nblk = a.nblk, ldw = 2 * nb;
    const int64_t te = int64_t(nb) * nb;
    zd *W = pole_window(a.window, pole, buf, nb);
    zd *Wn = pole_window(a.window, pole, buf ^ 1, nb);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int R = (k + 1 < nblk) ? 2 * nb : nb;
    const int cols = min(3 * nb, (nblk - k) * nb);       // window columns that exist
    const bool fin = (c0 + SW == nb);
    const int nleft = fin ? nb : c0;
    const int right0 = fin ? nb : c0 + SW;
    const int total = nleft + 3 * nb - right0;
    extern __shared__ unsigned char smem_raw[];
    zd *Ls = reinterpret_cast<zd *>(smem_raw);            // [SW][2nb]
    int *sp = reinterpret_cast<int *>(Ls + SW * ldw);     // [2nb]
    const int32_t *spg = a.subperm + int64_t(pole) * 2 * nb;
    for (int r = tid; r < R; r += kFacThreads) sp[r] = spg[r];
    const bool need_l = int(blockIdx.x) * kFacWaves + kFacWaves - 1 >= nleft;
    if (need_l) {
        // L of the sub-panel, rows c0..R-1 (rows above are not read)
        const int rr = R - c0, tot = rr * SW;
        for (int e0 = tid; e0 < tot; e0 += 4 * kFacThreads) {
            zd t[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int e = e0 + i * kFacThreads;
                t[i] = (e < tot) ? W[c0 + e % rr + int64_t(c0 + e / rr) * ldw] : zmake(0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int e = e0 + i * kFacThreads;
                if (e < tot) Ls[(e / rr) * ldw + c0 + e % rr] = t[i];
            }
        }
    }
    __syncthreads();
    const int slot = blockIdx.x * kFacWaves + wave;
    zd *T0 = a.tiles + tile_index(pole, k, 0, nblk, te);
    zd *T1 = T0 + te, *T2 = T1 + te, *T3 = T2 + te, *T4 = T3 + te;
    if (slot < total) {
        zd v[NS];
        if (slot < nleft) {
            const int col = slot;
            const bool perm_it = col < c0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                int r = lane + 64 * s;
                v[s] = (r < R) ? W[(perm_it ? sp[r] : r) + int64_t(col) * ldw] : zmake(0, 0);
            }
            if (fin) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int r = lane + 64 * s;
                    if (r < nb) { T0[r + int64_t(col) * nb] = v[s]; T2[r + int64_t(col) * nb] = v[s]; }
                    else if (r < 2 * nb) T1[(r - nb) + int64_t(col) * nb] = (r < R) ? v[s] : zmake(0, 0);
                }
            } else if (perm_it) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int r = lane + 64 * s;
                    if (r < R) W[r + int64_t(col) * ldw] = v[s];
                }
            }
        } else {
            const int col = right0 + (slot - nleft);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                int r = lane + 64 * s;
                v[s] = (r < R && col < cols) ? W[sp[r] + int64_t(col) * ldw] : zmake(0, 0);
            }
            const int sl = c0 >> 6, base = c0 & 63;
            zd vt = v[0];
#pragma unroll
            for (int s = 1; s < NS; ++s) if (s == sl) vt = v[s];
            for (int q = 0; q < SW; ++q) {
                const zd u = lane_bcast(vt, base + q);
                if (lane > base + q && lane < base + SW) zfms(vt, Ls[q * ldw + sl * 64 + lane], u);
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) if (s == sl) v[s] = vt;
            for (int q = 0; q < SW; ++q) {
                const zd u = lane_bcast(vt, base + q);
                const zd *lq = Ls + q * ldw;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int r = lane + 64 * s;
                    if (r >= c0 + SW && r < R) zfms(v[s], lq[r], u);
                }
            }
            if (fin) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int r = lane + 64 * s;
                    if (r < nb) {
                        if (col < 2 * nb) T3[r + int64_t(col - nb) * nb] = v[s];
                        else T4[r + int64_t(col - 2 * nb) * nb] = v[s];
                    } else if (r < R && k + 1 < nblk) {
                        Wn[(r - nb) + int64_t(col - nb) * ldw] = v[s];
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int r = lane + 64 * s;
                    if (r < R) W[r + int64_t(col) * ldw] = v[s];
                }
            }
        }
    }
    // last sub-step: next window's last column block of the top half is zero, its
    // bottom half is the prepared row block k+2 (column 0 = window column 0)
    if (fin && k + 1 < nblk) {
        const int64_t nthr = int64_t(gridDim.x) * kFacThreads;
        const int64_t gid = int64_t(blockIdx.x) * kFacThreads + tid;
        for (int64_t e = gid; e < te; e += nthr) {
            int r = int(e % nb), c = int(e / nb);
            Wn[r + int64_t(2 * nb + c) * ldw] = zmake(0, 0);
        }
        const int64_t tot = 3 * te;
        const zd *Pb = a.rows + (int64_t(pole) * nblk + (k + 2)) * tot;
        const bool have = k + 2 < nblk;
        for (int64_t e0 = gid; e0 < tot; e0 += 4 * nthr) {
            zd t[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t e = e0 + i * nthr;
                t[i] = (have && e < tot) ? Pb[e] : zmake(0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t e = e0 + i * nthr;
                if (e < tot) Wn[nb + int(e % nb) + (e / nb) * ldw] = t[i];
            }
        }
    }
}

// In-place inversion of the diagonal triangles, one workgroup per (block, pole,
// triangle).  blockIdx.z == 0: unit lower part of Linv slot; == 1: upper part of
// the Uinv slot.  Columns are done in groups of CG held in LDS; a column of the
// inverse only depends on entries of the triangle to its right (lower) or left
// (upper), so groups are processed left-to-right (lower) or right-to-left
// (upper) and written back in place.
template <int CG>
__global__ __launch_bounds__(kThreads) void tri_inverse_kernel(zd *tiles, int nb, int nblk) {
    constexpr int NPART = kThreads / CG;       // threads per column (same wave)
    const int k = blockIdx.x, pole = blockIdx.y, upper = blockIdx.z;
    const int64_t te = int64_t(nb) * nb;
    zd *T = tiles + tile_index(pole, k, upper ? 2 : 0, nblk, te);
    extern __shared__ unsigned char smem_raw[];
    zd *X = reinterpret_cast<zd *>(smem_raw);        // [nb][CG]
    const int tid = threadIdx.x;
    const int cl = tid / NPART, part = tid % NPART;  // parts of a column share a wave
    const int ngroups = (nb + CG - 1) / CG;
    for (int gi = 0; gi < ngroups; ++gi) {
        const int g = upper ? (ngroups - 1 - gi) : gi;
        const int c0 = g * CG;
        const int c = c0 + cl;
        for (int e = tid; e < nb * CG; e += kThreads) X[e] = zmake(0, 0);
        __syncthreads();
        if (!upper) {
            for (int r = c0; r < nb; ++r) {
                // X[r][c] = delta - sum_{b=c0}^{r-1} L[r][b] X[b][c]
                zd acc = zmake(0, 0);
                for (int b = c0 + part; b < r; b += NPART)
                    zfma(acc, T[r + int64_t(b) * nb], X[b * CG + cl]);
                for (int off = NPART / 2; off > 0; off >>= 1) {
                    acc.x += __shfl_xor(acc.x, off, 64);
                    acc.y += __shfl_xor(acc.y, off, 64);
                }
                if (part == 0 && c < nb && r >= c)
                    X[r * CG + cl] = (r == c) ? zmake(1.0, 0.0) : zmake(-acc.x, -acc.y);
                __syncthreads();
            }
        } else {
            const int rtop = min(nb, c0 + CG) - 1;
            for (int r = rtop; r >= 0; --r) {
                // X[r][c] = (delta - sum_{b=r+1}^{c0+CG-1} U[r][b] X[b][c]) / U[r][r]
                zd acc = zmake(0, 0);
                for (int b = r + 1 + part; b <= rtop; b += NPART)
                    zfma(acc, T[r + int64_t(b) * nb], X[b * CG + cl]);
                for (int off = NPART / 2; off > 0; off >>= 1) {
                    acc.x += __shfl_xor(acc.x, off, 64);
                    acc.y += __shfl_xor(acc.y, off, 64);
                }
                if (part == 0 && c < nb && r <= c) {
                    zd num = zsub((r == c) ? zmake(1.0, 0.0) : zmake(0, 0), acc);
                    zd d = T[r + int64_t(r) * nb];
                    X[r * CG + cl] = (zabs2(d) > 0.0) ? zdiv(num, d) : zmake(0, 0);
                }
                __syncthreads();
            }
        }
        // write the group back (whole columns: zeros outside the triangle)
        for (int e = tid; e < nb * CG; e += kThreads) {
            int r = e % nb, cc = e / nb;
            if (c0 + cc < nb) T[r + int64_t(c0 + cc) * nb] = X[r * CG + cc];
        }
        __syncthreads();
    }
}

// Register version for NB = 64 or 128: thread (row i = tid % NB, group g = tid / NB)
// holds columns g CPT .. g CPT + CPT - 1 of row i of X, which starts as the identity.
// Right-looking substitution: at step r (lower: r = 0 .. NB-1; upper: r = NB-1 .. 0) the
// owners of row r finish it (upper: scale by 1 / U_rr) and publish it in LDS (double
// buffered by step parity: one barrier per step), and every row still to be reached
// subtracts T_ir times it.  Column r of the triangle is read coalesced, eight steps
// of it at a time.  Row r of X is zero outside the triangle, so the update is taken
// by every row (times zero where it does not apply).
template <int NB>
__global__ __launch_bounds__(4 * NB) void tri_inverse_reg_kernel(zd *tiles, int nblk) {
    constexpr int CPT = NB / 4, STEPB = 8;
    const int k = blockIdx.x, pole = blockIdx.y, upper = blockIdx.z;
    constexpr int64_t te = int64_t(NB) * NB;
    zd *T = tiles + tile_index(pole, k, upper ? 2 : 0, nblk, te);
    const int tid = threadIdx.x, i = tid % NB, g = tid / NB, c0 = g * CPT;
    __shared__ zd xrow[2][NB];
    __shared__ zd rdiag[NB];
    zd a[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) a[q] = zmake(c0 + q == i ? 1.0 : 0.0, 0.0);
    if (upper && tid < NB) {
        const zd d = T[tid + int64_t(tid) * NB];
        const double s2 = zabs2(d);
        rdiag[tid] = (s2 > 0.0) ? zmake(d.x / s2, -d.y / s2) : zmake(0, 0);
    }
    __syncthreads();
    for (int s0 = 0; s0 < NB; s0 += STEPB) {
        zd tcol[STEPB];
#pragma unroll
        for (int u = 0; u < STEPB; ++u) {
            const int r = upper ? NB - 1 - (s0 + u) : s0 + u;
            const bool reach = upper ? (i < r) : (i > r);
            tcol[u] = reach ? T[i + int64_t(r) * NB] : zmake(0, 0);
        }
#pragma unroll
        for (int u = 0; u < STEPB; ++u) {
            const int r = upper ? NB - 1 - (s0 + u) : s0 + u;
            const int par = u & 1;
            if (i == r) {
                if (upper) {
                    const zd rr = rdiag[r];
#pragma unroll
                    for (int q = 0; q < CPT; ++q) a[q] = zmul(a[q], rr);
                }
#pragma unroll
                for (int q = 0; q < CPT; ++q) xrow[par][c0 + q] = a[q];
            }
            __syncthreads();
            // row r of X is zero left of r (upper) or right of r (lower): groups whose
            // columns all lie there skip the update (a group is whole waves)
            const bool live = upper ? (c0 + CPT - 1 >= r) : (c0 <= r);
            if (live) {
#pragma unroll
                for (int q = 0; q < CPT; ++q) zfms(a[q], tcol[u], xrow[par][c0 + q]);
            }
        }
    }
    __syncthreads();                       // every read of the triangle is done
#pragma unroll
    for (int q = 0; q < CPT; ++q) T[i + int64_t(c0 + q) * NB] = a[q];
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
struct SolveArgs {
    int n, nb, nblk, p;
    int ncols;               // total right-hand sides
    const zd *X; int64_t ldx;        // right-hand sides (before B)
    const zd *bdiag;                 // diagonal of B, or null (then X already holds B X)
    const void *tiles;               // factor tiles, complex128 or complex64
    const int32_t *perm;
    const zd *weights;               // w_i per pole
    const zd *colw;                  // or null: weight per pole and column, [pole][ncols]
    void *ypart;             // [pole][npad x ncols]  forward results (tile precision)
    zd *xpart;               // [pole][npad x ncols]  weight * K_i^{-1} B X
    int64_t npad;
    int64_t x_pole_stride;   // 0: one right-hand side block for all poles; else pole i's
                             // block starts at X + i * x_pole_stride (refinement residuals)
    int unit_weight;         // 1: no pole weight (the solution of K_i d = r itself)
    int accumulate;          // 1: xpart += solution (refinement correction), else xpart =
};

// complex64 helpers for the single-precision tiles
__device__ inline zf fmake(float re, float im) { zf r; r.x = re; r.y = im; return r; }
__device__ inline void zfma(zf &acc, zf a, zf b) {
    acc.x = fmaf(a.x, b.x, acc.x); acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y); acc.y = fmaf(a.y, b.x, acc.y);
}
__device__ inline zf zsub(zf a, zf b) { return fmake(a.x - b.x, a.y - b.y); }
template <typename CT> __device__ inline CT czero() { CT z; z.x = 0; z.y = 0; return z; }
template <typename CT> __device__ inline CT from_zd(zd v);
template <> __device__ inline zd from_zd<zd>(zd v) { return v; }
template <> __device__ inline zf from_zd<zf>(zd v) { return fmake(float(v.x), float(v.y)); }
__device__ inline zd to_zd(zd v) { return v; }
__device__ inline zd to_zd(zf v) { return zmake(double(v.x), double(v.y)); }

// Solve kernel.  One workgroup of kSolveThreads threads owns one pole and a slice
// of CW right-hand sides and runs the whole forward and backward sweep as nb x nb
// tile products out = T v.  Tiles are stored whole (the inverted triangles carry
// explicit zeros); the parts of a thread's piece that are structurally zero in a
// triangular tile are skipped at compile time, so every thread issues the same
// loads on every path.  Layout (template on the tile size NB, a power of two):
// the NB rows are spread over SLOTS row slots with R rows each (rows s, s + SLOTS,
// ...), the columns over G lanes (column k = j G + g), so a thread holds an R x KL
// piece of the tile and each LDS read of v feeds R multiply-adds; the G partial sums
// of a row are combined with cross-lane shuffles.  Lanes are slot-fastest, so one
// load instruction reads G runs of 64/G consecutive rows of a tile column.
//
// The tile reads of the whole solve form one fixed sequence -- forward: Linv_k,
// L21_k per block; backward: U1_k, U2_k, Uinv_k -- independent of the data, so
// they are software-pipelined: a thread's piece of a tile is split into NBAT
// batches held in two register buffers, and as soon as a batch has been consumed
// the batch two places further down the sequence is requested, so the next
// product's loads are in flight across the reductions and barriers of the current
// one.  Where registers allow, the entries of v that a batch multiplies are read
// from LDS one batch ahead too, so the multiply-adds do not wait on LDS latency.
// The workgroups of a pole also touch the next block's tiles so that they are in L2.
constexpr int kSolveThreads = 512;

template <int NB, int NT = kSolveThreads>
struct SolveShape {
    static constexpr int R = NB >= 64 ? NB / 64 : 1;                  // rows per thread
    static constexpr int SLOTS = NB / R;
    static constexpr int G0 = NT / SLOTS;
    static constexpr int G = G0 < NB / 2 ? G0 : NB / 2;               // lanes per slot
    static constexpr int KL = NB / G;                                 // columns per thread
    static constexpr int L = R * KL;                                  // tile elements per thread
    static constexpr int S = L / 2 < 8 ? L / 2 : 8;                   // batch size
    static constexpr int NBAT = L / S;                                // batches per tile (even)
    static constexpr int RPW = 64 / G;                                // slots per wave
    static constexpr int ACTIVE = SLOTS * G;                          // threads with rows
    static_assert(NBAT % 2 == 0 && S >= 1 && ACTIVE <= NT, "solve shape");
};

// Shape of a tile: full, or triangular with structural zeros (Linv and U2 lower,
// Uinv upper).  Element (q, j) of a thread's piece covers rows [q SLOTS, (q+1) SLOTS)
// and columns [j G, j G + G) of the tile; it is skipped when all of it is zero.
enum : int { kFull = 0, kLower = 1, kUpper = 2 };

template <int NB, int NT, int SHAPE>
__device__ constexpr bool piece_zero(int q, int j) {
    using SH = SolveShape<NB, NT>;
    return SHAPE == kLower ? ((q + 1) * SH::SLOTS - 1 < j * SH::G)
         : SHAPE == kUpper ? (q * SH::SLOTS > j * SH::G + SH::G - 1) : false;
}

// Load batch b of this thread's piece of tile T (thread corner tp = T + slot + g NB;
// the element offsets are compile-time constants).
template <int NB, int NT, int SHAPE, typename CT>
__device__ __attribute__((always_inline)) inline void issue_batch(const CT *tp, int b,
                                                                  CT (&t)[SolveShape<NB, NT>::S]) {
    using SH = SolveShape<NB, NT>;
#pragma unroll
    for (int e = 0; e < SH::S; ++e) {
        const int E = b * SH::S + e, j = E / SH::R, q = E % SH::R;
        if (!piece_zero<NB, NT, SHAPE>(q, j)) t[e] = tp[SH::SLOTS * q + j * SH::G * NB];
    }
}

// acc[q][c] += sum over batch b of a tile of T[row_q, k] v[k, c]
template <int CW, int NB, int NT, int SHAPE, typename CT>
__device__ __attribute__((always_inline)) inline void consume(int g, int b,
                                                              const CT (&t)[SolveShape<NB, NT>::S],
                                                              const CT *v,
                                                              CT (&acc)[SolveShape<NB, NT>::R][CW]) {
    using SH = SolveShape<NB, NT>;
#pragma unroll
    for (int e = 0; e < SH::S; ++e) {
        const int E = b * SH::S + e, j = E / SH::R, q = E % SH::R;
        if (piece_zero<NB, NT, SHAPE>(q, j)) continue;
        const CT *vr = v + (j * SH::G + g) * CW;
#pragma unroll
        for (int c = 0; c < CW; ++c) zfma(acc[q][c], t[e], vr[c]);
    }
}

// One tile product of the stream: consume the tile of shape SC held in bufA / bufB
// (even / odd batches) and request, batch by batch, the rest of it and then the
// first batches of the next tile, read as shape SN.  A consumer never uses an
// element its producer skipped: SN is the next tile's shape or kFull.
template <int CW, int NB, int NT, int SC, int SN, typename CT>
__device__ __attribute__((always_inline)) inline void run_phase(
        int g, CT (&bufA)[SolveShape<NB, NT>::S], CT (&bufB)[SolveShape<NB, NT>::S],
        CT (&acc)[SolveShape<NB, NT>::R][CW], const CT *v, const CT *tcur, const CT *tnext) {
    using SH = SolveShape<NB, NT>;
#pragma unroll
    for (int bp = 0; bp < SH::NBAT; bp += 2) {
        consume<CW, NB, NT, SC, CT>(g, bp, bufA, v, acc);
        if (bp + 2 < SH::NBAT) issue_batch<NB, NT, SC, CT>(tcur, bp + 2, bufA);
        else issue_batch<NB, NT, SN, CT>(tnext, bp + 2 - SH::NBAT, bufA);
        consume<CW, NB, NT, SC, CT>(g, bp + 1, bufB, v, acc);
        if (bp + 3 < SH::NBAT) issue_batch<NB, NT, SC, CT>(tcur, bp + 3, bufB);
        else issue_batch<NB, NT, SN, CT>(tnext, bp + 3 - SH::NBAT, bufB);
    }
}

// the entries of v that batch b of a tile piece multiplies: columns j G + g for the
// batch's S / R values of j
template <int CW, int NB, int NT, typename CT>
__device__ __attribute__((always_inline)) inline void load_v(
        int g, int b, const CT *v, CT (&vb)[SolveShape<NB, NT>::S / SolveShape<NB, NT>::R][CW]) {
    using SH = SolveShape<NB, NT>;
    constexpr int JB = SH::S / SH::R;
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
        const CT *vr = v + ((b * SH::S) / SH::R + jj) * SH::G * CW + g * CW;
#pragma unroll
        for (int c = 0; c < CW; ++c) vb[jj][c] = vr[c];
    }
}

// consume with the batch's entries of v already in registers
template <int CW, int NB, int NT, int SHAPE, typename CT>
__device__ __attribute__((always_inline)) inline void consume_v(
        int b, const CT (&t)[SolveShape<NB, NT>::S],
        const CT (&vb)[SolveShape<NB, NT>::S / SolveShape<NB, NT>::R][CW],
        CT (&acc)[SolveShape<NB, NT>::R][CW]) {
    using SH = SolveShape<NB, NT>;
#pragma unroll
    for (int e = 0; e < SH::S; ++e) {
        const int E = b * SH::S + e, j = E / SH::R, q = E % SH::R;
        if (piece_zero<NB, NT, SHAPE>(q, j)) continue;
        const int jj = j - (b * SH::S) / SH::R;
#pragma unroll
        for (int c = 0; c < CW; ++c) zfma(acc[q][c], t[e], vb[jj][c]);
    }
}

// run_phase with the entries of v read one batch ahead into two register sets
template <int CW, int NB, int NT, int SC, int SN, typename CT>
__device__ __attribute__((always_inline)) inline void run_phase_vpre(
        int g, CT (&bufA)[SolveShape<NB, NT>::S], CT (&bufB)[SolveShape<NB, NT>::S],
        CT (&acc)[SolveShape<NB, NT>::R][CW], const CT *v, const CT *tcur, const CT *tnext) {
    using SH = SolveShape<NB, NT>;
    constexpr int JB = SH::S / SH::R;
    static_assert(SH::S % SH::R == 0, "batch covers whole columns");
    CT vA[JB][CW], vB[JB][CW];
    load_v<CW, NB, NT, CT>(g, 0, v, vA);
    load_v<CW, NB, NT, CT>(g, 1, v, vB);
#pragma unroll
    for (int bp = 0; bp < SH::NBAT; bp += 2) {
        consume_v<CW, NB, NT, SC, CT>(bp, bufA, vA, acc);
        if (bp + 2 < SH::NBAT) issue_batch<NB, NT, SC, CT>(tcur, bp + 2, bufA);
        else issue_batch<NB, NT, SN, CT>(tnext, bp + 2 - SH::NBAT, bufA);
        if (bp + 2 < SH::NBAT) load_v<CW, NB, NT, CT>(g, bp + 2, v, vA);
        consume_v<CW, NB, NT, SC, CT>(bp + 1, bufB, vB, acc);
        if (bp + 3 < SH::NBAT) issue_batch<NB, NT, SC, CT>(tcur, bp + 3, bufB);
        else issue_batch<NB, NT, SN, CT>(tnext, bp + 3 - SH::NBAT, bufB);
        if (bp + 3 < SH::NBAT) load_v<CW, NB, NT, CT>(g, bp + 3, v, vB);
    }
}

// The tile products of the solve: the v-prefetching form where its two register
// sets fit beside the accumulators (complex128 up to two columns, complex64 up to
// four), the plain form otherwise.
template <int CW, int NB, int NT, int SC, int SN, typename CT>
__device__ __attribute__((always_inline)) inline void tile_product(
        int g, CT (&bufA)[SolveShape<NB, NT>::S], CT (&bufB)[SolveShape<NB, NT>::S],
        CT (&acc)[SolveShape<NB, NT>::R][CW], const CT *v, const CT *tcur, const CT *tnext) {
    if constexpr (CW * sizeof(CT) <= 32)
        run_phase_vpre<CW, NB, NT, SC, SN, CT>(g, bufA, bufB, acc, v, tcur, tnext);
    else
        run_phase<CW, NB, NT, SC, SN, CT>(g, bufA, bufB, acc, v, tcur, tnext);
}

template <int CW, int NB, int NT, typename CT>
__device__ inline void reduce_rows(CT (&acc)[(SolveShape<NB, NT>::R)][CW]) {
    using SH = SolveShape<NB, NT>;
#pragma unroll
    for (int off = SH::G / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < SH::R; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                acc[q][c].x += __shfl_xor(acc[q][c].x, off * SH::RPW, 64);
                acc[q][c].y += __shfl_xor(acc[q][c].y, off * SH::RPW, 64);
            }
    }
}

template <int CW, int NB, int NT, typename CT>
__global__ __launch_bounds__(NT) void band_solve_kernel(SolveArgs a) {
    using SH = SolveShape<NB, NT>;
    constexpr int R = SH::R;
    const int p = a.p;
    const int pole = blockIdx.x % p;             // slices of one pole share an XCD
    const int slice = blockIdx.x / p;
    const int c0 = slice * CW;
    if (c0 >= a.ncols) return;
    const int ncw = min(CW, a.ncols - c0);
    const int nblk = a.nblk;
    constexpr int64_t te = int64_t(NB) * NB;
    const int tid = threadIdx.x;
    const zd wgt = a.weights[pole];
    const int wave = tid / 64, lane = tid % 64;
    const int g = lane / SH::RPW;
    const int slot_raw = wave * SH::RPW + lane % SH::RPW;
    const bool active = tid < SH::ACTIVE;
    const int slot = active ? slot_raw : 0;                  // idle threads read row 0
    const bool writer = active && g == 0;

    // The 256-thread form (eight columns at tile 256) keeps its forward window in three
    // nb-row buffers (see the forward sweep): a second 2nb-row window would not fit the
    // LDS.  Its ring of backward blocks reuses those buffers.
    constexpr bool inplace = NT < kSolveThreads;
    constexpr bool late_y = CW >= 8;              // see the backward sweep
    extern __shared__ unsigned char smem_raw[];
    CT *win = reinterpret_cast<CT *>(smem_raw);   // [2NB][CW] (256 threads: [3][NB][CW])
    CT *win2 = inplace ? win : win + 2 * NB * CW; // [2NB][CW]: the permuted window
    CT *ybuf = inplace ? win + 3 * NB * CW : win2 + 2 * NB * CW;   // [NB][CW]
    CT *ring = inplace ? win : ybuf + NB * CW;    // [3][NB][CW]

    CT *yp = static_cast<CT *>(a.ypart) + int64_t(pole) * a.npad * a.ncols;
    zd *xp = a.xpart + int64_t(pole) * a.npad * a.ncols;
    const CT *tiles = static_cast<const CT *>(a.tiles) + int64_t(pole) * nblk * 5 * te;
    const int32_t *perm = a.perm + int64_t(pole) * nblk * 2 * NB;

    // tile of block k, slot t (0 Linv, 1 L21, 2 Uinv, 3 U1, 4 U2), at this thread's corner
    const int64_t corner = slot + int64_t(g) * NB;
    auto tile_at = [&](int k, int t) __attribute__((always_inline)) {
        return tiles + (int64_t(k) * 5 + t) * te + corner;
    };

    // L2 prefetch: the workgroups of this pole that share an XCD (workgroups are
    // dealt to the 8 XCDs round-robin) split the next step's tiles between them and
    // each thread touches one 128-byte line.
    const int nslices = (a.ncols + CW - 1) / CW;
    const int spread = (8 % p == 0) ? 8 / p : 1;          // XCDs one pole is spread over
    const int prank = slice / spread;
    const int pcount = (nslices + spread - 1) / spread;
    double sink = 0.0;
    auto touch = [&](const CT *base, int64_t elems) __attribute__((always_inline)) {
        constexpr int64_t kLine = 128 / sizeof(CT);         // elements per 128-byte line
        const int64_t lines = (elems + kLine - 1) / kLine;
        const int64_t per = (lines + pcount - 1) / pcount;
        const int64_t ln = int64_t(prank) * per + tid;
        const bool ok = tid < per && ln < lines;
        sink += double(base[ok ? ln * kLine : 0].x);
    };

    // right-hand sides: rows of block blk, element e of the [NB][CW] block
    const zd *Xp = a.X + int64_t(pole) * a.x_pole_stride;
    constexpr int RPT = (NB * CW + NT - 1) / NT;
    CT pre[RPT];
    auto prefetch_rhs = [&](int blk) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int e = tid + q * NT;
            const int r = e / CW, c = e % CW;
            const int64_t row = int64_t(blk) * NB + r;
            const bool ok = blk < nblk && e < NB * CW && row < a.n && c < ncw;
            zd x = Xp[ok ? row + int64_t(c0 + c) * a.ldx : 0];
            if (a.bdiag) x = zmul(a.bdiag[ok ? row : 0], x);
            pre[q] = ok ? from_zd<CT>(x) : czero<CT>();
        }
    };
    auto store_rhs = [&](CT *dst) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int e = tid + q * NT;
            if (e < NB * CW) dst[e] = pre[q];
        }
    };

    // the pipelined tile stream: bufA / bufB hold the even / odd batches of the tile
    // being consumed; each consumed batch is replaced by the one two places further
    // down the sequence (the same tile, or the next one)
    CT bufA[SH::S], bufB[SH::S];
    issue_batch<NB, NT, kFull, CT>(tile_at(0, 0), 0, bufA);
    issue_batch<NB, NT, kFull, CT>(tile_at(0, 0), 1, bufB);
    CT acc[R][CW];
    auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) acc[q][c] = czero<CT>();
    };

    // ---------------- forward sweep
    // Window of step k: [t_k; b_{k+1}], permuted by P_k.  The 512-thread form keeps it in
    // win (2nb rows) and its permuted copy in win2.  The 256-thread form has three
    // nb-row buffers in turn: t_k, b_{k+1} and a free one, which receives the permuted top
    // half (w_top) and, once that has been consumed, t_{k+1}; the bottom half (w_bot) is
    // read through the permutation where it is used.
    constexpr int GROWS = inplace ? 1 : 2;                 // window halves gathered
    constexpr int GPT = (GROWS * NB * CW + NT - 1) / NT;  // gathered elements per thread
    auto third = [&](int i) __attribute__((always_inline)) {
        return win + ((i % 3 + 3) % 3) * NB * CW;
    };
    prefetch_rhs(0);
    store_rhs(win);                                      // b_0 (the t-buffer of step 0)
    prefetch_rhs(1);
    for (int k = 0; k < nblk; ++k) {
        const bool last = (k + 1 == nblk);
        CT *tb = inplace ? third(-k) : win;                  // t_k
        CT *bb = inplace ? third(1 - k) : win + NB * CW;     // b_{k+1}
        CT *gb = inplace ? third(2 - k) : win2;              // permuted window
        if (!last) store_rhs(bb);                            // b_{k+1}
        prefetch_rhs(k + 2);                                 // b_{k+2}, used next step
        touch(tiles + int64_t(min(k + 1, nblk - 1)) * 5 * te, 2 * te);   // Linv, L21 of step k+1
        const int rows = (last || inplace) ? NB : 2 * NB;
        const int32_t *pk = perm + int64_t(k) * 2 * NB;
        int pr[GPT];
#pragma unroll
        for (int q = 0; q < GPT; ++q) pr[q] = pk[min(tid + q * NT, rows * CW - 1) / CW];
        int pb[inplace ? R : 1];                             // window rows of w_bot (writers)
        if constexpr (inplace) {
#pragma unroll
            for (int q = 0; q < R; ++q) pb[q] = (writer && !last) ? pk[NB + slot + SH::SLOTS * q] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < GPT; ++q) {
            const int e = min(tid + q * NT, rows * CW - 1);  // past the end: same value again
            const int src = pr[q];
            if constexpr (inplace)
                gb[e] = src < NB ? tb[src * CW + e % CW] : bb[(src - NB) * CW + e % CW];
            else
                gb[e] = win[src * CW + e % CW];
        }
        __syncthreads();
        zero_acc();
        tile_product<CW, NB, NT, kLower, kFull, CT>(g, bufA, bufB, acc, gb, tile_at(k, 0),
                                                tile_at(k, 1));          // y_k = Linv w_top
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    ybuf[row * CW + c] = acc[q][c];
                    if (c < ncw) yp[int64_t(k) * NB + row + int64_t(c0 + c) * a.npad] = acc[q][c];
                }
            }
        }
        __syncthreads();
        zero_acc();
        // next: Linv_{k+1}, or U1 of the last block to start the backward sweep
        tile_product<CW, NB, NT, kFull, kFull, CT>(g, bufA, bufB, acc, ybuf, tile_at(k, 1),
                                               last ? tile_at(k, 3) : tile_at(k + 1, 0));   // t_{k+1} = w_bot - L21 y_k
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer && !last) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
                if constexpr (inplace) {
                    const int src = pb[q];
                    const CT *wb = src < NB ? tb + src * CW : bb + (src - NB) * CW;
#pragma unroll
                    for (int c = 0; c < CW; ++c) gb[row * CW + c] = zsub(wb[c], acc[q][c]);
                } else {
#pragma unroll
                    for (int c = 0; c < CW; ++c) win[row * CW + c] = zsub(win2[(NB + row) * CW + c], acc[q][c]);
                }
            }
        }
        __syncthreads();
    }
    // ---------------- backward sweep
    for (int e = tid; e < 3 * NB * CW; e += NT) ring[e] = czero<CT>();
    touch(tiles + int64_t(nblk - 1) * 5 * te + 2 * te, 3 * te);
    CT ynext[R][CW];
    auto load_y = [&](int k, CT (&dst)[R][CW]) {
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const bool ok = writer && k >= 0 && c < ncw;
                const CT x = yp[ok ? int64_t(k) * NB + slot + SH::SLOTS * q + int64_t(c0 + c) * a.npad : 0];
                dst[q][c] = ok ? x : czero<CT>();
            }
    };
    // y_k is read one step ahead, or (eight columns, whose 4 x 8 blocks would take two
    // register sets) at the start of its own step, in flight during the first products
    if constexpr (!late_y) load_y(nblk - 1, ynext);
    __syncthreads();
    for (int k = nblk - 1; k >= 0; --k) {
        CT *xk = ring + (k % 3) * NB * CW;
        const CT *xk1 = ring + ((k + 1) % 3) * NB * CW;
        const CT *xk2 = ring + ((k + 2) % 3) * NB * CW;
        CT y[R][CW];
        if constexpr (late_y) {
            load_y(k, y);
        } else {
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int c = 0; c < CW; ++c) y[q][c] = ynext[q][c];
            load_y(k - 1, ynext);                                   // y_{k-1}, used next step
        }
        touch(tiles + int64_t(max(k - 1, 0)) * 5 * te + 2 * te, 3 * te);   // Uinv, U1, U2 of k-1
        // v = y_k - U1 x_{k+1} - U2 x_{k+2}
        zero_acc();
        tile_product<CW, NB, NT, kFull, kLower, CT>(g, bufA, bufB, acc, xk1, tile_at(k, 3),
                                                tile_at(k, 4));
        tile_product<CW, NB, NT, kLower, kUpper, CT>(g, bufA, bufB, acc, xk2, tile_at(k, 4),
                                                 tile_at(k, 2));
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) ybuf[row * CW + c] = zsub(y[q][c], acc[q][c]);
            }
        }
        __syncthreads();
        zero_acc();
        tile_product<CW, NB, NT, kUpper, kFull, CT>(g, bufA, bufB, acc, ybuf, tile_at(k, 2),
                                                tile_at(max(k - 1, 0), 3));   // x_k = Uinv v
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    xk[row * CW + c] = acc[q][c];
                    if (c < ncw) {
                        const zd wc = a.unit_weight ? zmake(1.0, 0.0)
                                    : a.colw ? a.colw[int64_t(pole) * a.ncols + c0 + c] : wgt;
                        zd *dst = xp + int64_t(k) * NB + row + int64_t(c0 + c) * a.npad;
                        const zd val = zmul(wc, to_zd(acc[q][c]));
                        *dst = a.accumulate ? zadd(*dst, val) : val;
                    }
                }
            }
        }
        __syncthreads();
    }
    // keep the prefetch loads alive without storing anything real (n is never negative)
    if (a.n < 0) ybuf[0] = from_zd<CT>(zmake(sink, 0.0));
}

// Conjugate-transposed solve, K^H x = d, with the factors of K (the differentiation
// form: left eigenvectors from the adjoint pencil (A^H, B^H), whose shifted matrices
// at the conjugate poles are the K_i^H).  K = Lhat U, where Lhat^{-1} is the product
// of the block steps M_k = [Linv_k, 0; -L21_k Linv_k, I] P_k acting on row blocks
// (k, k+1), so K^H = U^H Lhat^H and
//   U^H sweep (k = 0 .. nblk-1):  v_k = Uinv_k^H (d_k - U1_{k-1}^H v_{k-1} - U2_{k-2}^H v_{k-2})
//   Lhat^H sweep (k = nblk-1 .. 0), with b the current row block k+1:
//       a' = Linv_k^H (v_k - L21_k^H b),   [block k; block k+1] = P_k^T [a'; b],
//   after which block k+1 is final.  The tiles read here are the conjugate transposes
// of the factor's tiles (slot t holds T_t^H: Linv^H and U2^H upper, Uinv^H lower),
// made once from the factorization, so both sweeps are the same tile products as the
// plain solve.  One workgroup per (pole, slice of CW right-hand sides), as there.
template <int CW, int NB, int NT, typename CT>
__global__ __launch_bounds__(NT) void band_solve_adj_kernel(SolveArgs a) {
    using SH = SolveShape<NB, NT>;
    constexpr int R = SH::R;
    const int p = a.p;
    const int pole = blockIdx.x % p;
    const int slice = blockIdx.x / p;
    const int c0 = slice * CW;
    if (c0 >= a.ncols) return;
    const int ncw = min(CW, a.ncols - c0);
    const int nblk = a.nblk;
    constexpr int64_t te = int64_t(NB) * NB;
    const int tid = threadIdx.x;
    const zd wgt = a.weights[pole];
    const int wave = tid / 64, lane = tid % 64;
    const int g = lane / SH::RPW;
    const int slot_raw = wave * SH::RPW + lane % SH::RPW;
    const bool active = tid < SH::ACTIVE;
    const int slot = active ? slot_raw : 0;
    const bool writer = active && g == 0;

    extern __shared__ unsigned char smem_raw[];
    CT *ring = reinterpret_cast<CT *>(smem_raw);   // [3][NB][CW]: v_{k-2}, v_{k-1}, v_k
    CT *tb = ring + 3 * NB * CW;                   // [NB][CW]: right-hand side of a triangle
    CT *abuf = tb + NB * CW;                       // [NB][CW]: a' before the interchange
    CT *cbuf[2] = {abuf + NB * CW, abuf + 2 * NB * CW};   // [NB][CW] x 2: row block k+1

    CT *yp = static_cast<CT *>(a.ypart) + int64_t(pole) * a.npad * a.ncols;
    zd *xp = a.xpart + int64_t(pole) * a.npad * a.ncols;
    const CT *tiles = static_cast<const CT *>(a.tiles) + int64_t(pole) * nblk * 5 * te;
    const int32_t *perm = a.perm + int64_t(pole) * nblk * 2 * NB;
    const int64_t corner = slot + int64_t(g) * NB;
    auto tile_at = [&](int k, int t) __attribute__((always_inline)) {
        return tiles + (int64_t(k) * 5 + t) * te + corner;
    };

    constexpr int RPT = (NB * CW + NT - 1) / NT;
    CT pre[RPT];
    auto prefetch_rhs = [&](int blk) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int e = tid + q * NT;
            const int r = e / CW, c = e % CW;
            const int64_t row = int64_t(blk) * NB + r;
            const bool ok = blk < nblk && e < NB * CW && row < a.n && c < ncw;
            zd x = a.X[ok ? row + int64_t(c0 + c) * a.ldx : 0];
            if (a.bdiag) x = zmul(a.bdiag[ok ? row : 0], x);
            pre[q] = ok ? from_zd<CT>(x) : czero<CT>();
        }
    };
    CT bufA[SH::S], bufB[SH::S];
    issue_batch<NB, NT, kFull, CT>(tile_at(0, 3), 0, bufA);
    issue_batch<NB, NT, kFull, CT>(tile_at(0, 3), 1, bufB);
    CT acc[R][CW];
    auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) acc[q][c] = czero<CT>();
    };

    // ---------------- U^H sweep
    for (int e = tid; e < 3 * NB * CW; e += NT) ring[e] = czero<CT>();
    prefetch_rhs(0);
    for (int k = 0; k < nblk; ++k) {
        const bool last = (k + 1 == nblk);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int e = tid + q * NT;
            if (e < NB * CW) tb[e] = pre[q];             // d_k
        }
        prefetch_rhs(k + 1);
        __syncthreads();
        CT *vk = ring + (k % 3) * NB * CW;
        const CT *vk1 = ring + ((k + 2) % 3) * NB * CW;   // v_{k-1} (zero for k < 1)
        const CT *vk2 = ring + ((k + 1) % 3) * NB * CW;   // v_{k-2} (zero for k < 2)
        zero_acc();
        tile_product<CW, NB, NT, kFull, kUpper, CT>(g, bufA, bufB, acc, vk1, tile_at(max(k - 1, 0), 3),
                                                tile_at(max(k - 2, 0), 4));
        tile_product<CW, NB, NT, kUpper, kLower, CT>(g, bufA, bufB, acc, vk2, tile_at(max(k - 2, 0), 4),
                                                 tile_at(k, 2));
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) tb[row * CW + c] = zsub(tb[row * CW + c], acc[q][c]);
            }
        }
        __syncthreads();
        zero_acc();
        // next: U1_k^H, the first product of step k + 1, or L21^H of the last block
        tile_product<CW, NB, NT, kLower, kFull, CT>(g, bufA, bufB, acc, tb, tile_at(k, 2),
                                                last ? tile_at(nblk - 1, 1) : tile_at(k, 3));
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    vk[row * CW + c] = acc[q][c];
                    if (c < ncw) yp[int64_t(k) * NB + row + int64_t(c0 + c) * a.npad] = acc[q][c];
                }
            }
        }
        __syncthreads();
    }
    // ---------------- Lhat^H sweep
    for (int e = tid; e < NB * CW; e += NT) cbuf[0][e] = czero<CT>();
    CT ynext[R][CW];
    auto load_v = [&](int k, CT (&dst)[R][CW]) {
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const bool ok = writer && k >= 0 && c < ncw;
                const CT x = yp[ok ? int64_t(k) * NB + slot + SH::SLOTS * q + int64_t(c0 + c) * a.npad : 0];
                dst[q][c] = ok ? x : czero<CT>();
            }
    };
    load_v(nblk - 1, ynext);
    __syncthreads();
    int cb = 0;
    for (int k = nblk - 1; k >= 0; --k) {
        const CT *cur = cbuf[cb];
        CT *curn = cbuf[cb ^ 1];
        CT v[R][CW];
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) v[q][c] = ynext[q][c];
        load_v(k - 1, ynext);
        zero_acc();
        tile_product<CW, NB, NT, kFull, kUpper, CT>(g, bufA, bufB, acc, cur, tile_at(k, 1),
                                                tile_at(k, 0));           // L21_k^H b
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) tb[row * CW + c] = zsub(v[q][c], acc[q][c]);
            }
        }
        __syncthreads();
        zero_acc();
        tile_product<CW, NB, NT, kUpper, kFull, CT>(g, bufA, bufB, acc, tb, tile_at(k, 0),
                                                tile_at(max(k - 1, 0), 1));   // a' = Linv_k^H t
        reduce_rows<CW, NB, NT, CT>(acc);
        if (writer) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int row = slot + SH::SLOTS * q;
#pragma unroll
                for (int c = 0; c < CW; ++c) abuf[row * CW + c] = acc[q][c];
            }
        }
        __syncthreads();
        // [block k; block k+1] = P_k^T [a'; b]: window row i goes back to position perm[i]
        const int rows = (k + 1 == nblk) ? NB : 2 * NB;
        const int32_t *pk = perm + int64_t(k) * 2 * NB;
        for (int e = tid; e < rows * CW; e += NT) {
            const int i = e / CW, c = e % CW;
            const CT val = i < NB ? abuf[e] : cur[e - NB * CW];
            const int d = pk[i];
            if (d < NB) curn[d * CW + c] = val;
            else if (c < ncw)
                xp[int64_t(k + 1) * NB + (d - NB) + int64_t(c0 + c) * a.npad] = zmul(wgt, to_zd(val));
        }
        __syncthreads();
        cb ^= 1;
    }
    for (int e = tid; e < NB * CW; e += NT) {
        const int i = e / CW, c = e % CW;
        if (c < ncw) xp[i + int64_t(c0 + c) * a.npad] = zmul(wgt, to_zd(cbuf[cb][e]));
    }
}

// Conjugate transposes of the factor tiles of pole src_pole (one workgroup per
// (tile, block, destination pole)), through LDS in 32 x 32 pieces (whole tile below
// 32): dst(r, c) = conj(src(c, r)).
__global__ __launch_bounds__(256) void tiles_adjoint_kernel(const zd *src, zd *dst, int p, int nblk,
                                                            int nb) {
    const int t = blockIdx.x % 5, k = blockIdx.x / 5, pd = blockIdx.y;
    const int ps = p - 1 - pd;                 // the adjoint pole pd is the conjugate of pole ps
    const int64_t te = int64_t(nb) * nb;
    const zd *S = src + ((int64_t(ps) * nblk + k) * 5 + t) * te;
    zd *D = dst + ((int64_t(pd) * nblk + k) * 5 + t) * te;
    __shared__ zd tile[32][33];
    const int P = nb < 32 ? nb : 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;    // 32 x 8
    for (int bc = 0; bc < nb; bc += P)
        for (int br = 0; br < nb; br += P) {
            // read the piece at rows br.., columns bc.. of S (coalesced down the columns)
            for (int j = ty; j < P; j += 8)
                if (tx < P) tile[j][tx] = S[(br + tx) + int64_t(bc + j) * nb];
            __syncthreads();
            // write it transposed to rows bc.., columns br.. of D
            for (int j = ty; j < P; j += 8)
                if (tx < P) {
                    const zd v = tile[tx][j];
                    D[(bc + tx) + int64_t(br + j) * nb] = zmake(v.x, -v.y);
                }
            __syncthreads();
        }
}

// FP64 residual of the shifted solves for iterative refinement, every pole at once:
// res_i = w b - K_i x_i = w b - p_i B x_i + A x_i, with x_i = xpart[pole] (which holds
// w K_i^{-1} b from the complex64 solve) and b = B X (bdiag: diagonal B; rhsb: B X
// already formed; neither: b = X).  w is the pole weight, or the per-(pole, column)
// weight of the residual form (colw).  One thread per (row, column, pole).
__global__ void refine_residual_kernel(int n, int ncols, int p, int64_t npad, const zd *X, int64_t ldx,
                                       const zd *bdiag, const zd *rhsb, const int32_t *arow,
                                       const int32_t *acol, const zd *aval, const int32_t *brow,
                                       const int32_t *bcol, const zd *bval, const zd *poles,
                                       const zd *weights, const zd *colw, const zd *xpart, zd *res) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(n) * ncols;
    if (e >= per * p) return;
    const int pole = int(e / per);
    const int64_t rc = e % per;
    const int row = int(rc % n), c = int(rc / n);
    const zd *x = xpart + int64_t(pole) * npad * ncols + int64_t(c) * npad;
    zd b;
    if (rhsb) b = rhsb[row + int64_t(c) * npad];
    else {
        b = X[row + int64_t(c) * ldx];
        if (bdiag) b = zmul(bdiag[row], b);
    }
    const zd w = colw ? colw[int64_t(pole) * ncols + c] : weights[pole];
    zd r = zmul(w, b);
    zd bx = zmake(0, 0);
    for (int q = brow[row]; q < brow[row + 1]; ++q) zfma(bx, bval[q], x[bcol[q]]);
    zfms(r, poles[pole], bx);
    for (int q = arow[row]; q < arow[row + 1]; ++q) zfma(r, aval[q], x[acol[q]]);
    res[int64_t(pole) * npad * ncols + int64_t(c) * npad + row] = r;
}

// Z[:, c] = sum_pole xpart[pole][:, c]   (fixed order: deterministic)
__global__ void pole_sum_kernel(const zd *xpart, int p, int64_t npad, int64_t n, int ncols,
                                zd *Z, int64_t ldz) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    zd s = xpart[r + c * npad];
    for (int i = 1; i < p; ++i) s = zadd(s, xpart[int64_t(i) * npad * ncols + r + c * npad]);
    Z[r + c * ldz] = s;
}

}  // namespace

hipError_t launch_band_factor(const rf_plan &P, hipStream_t s) {
    FactorArgs a;
    a.n = int(P.n); a.nb = P.F.nb; a.nblk = P.F.nblk;
    a.arow = P.A.rowptr; a.acol = P.A.colind; a.aval = P.A.val;
    a.brow = P.B.rowptr; a.bcol = P.B.colind; a.bval = P.B.val;
    a.poles = P.d_poles; a.tiles = P.F.tiles; a.perm = P.F.perm; a.window = P.F.window;
    a.info = P.F.info;
    const int nb = a.nb;
    const int p = P.opts.p;
    // sub-steps of 32 columns when the trail kernel's L staging fits, else 16
    auto trail_lds = [&](int sw) {
        return size_t(sw) * 2 * nb * sizeof(zd) + size_t(2 * nb) * sizeof(int);
    };
    const int sw = (nb % 32 == 0 && trail_lds(32) <= size_t(P.max_lds)) ? 32 : 16;
    const int ns = (2 * nb + 63) / 64;
    if (trail_lds(sw) > size_t(P.max_lds) || nb > 256) return hipErrorInvalidValue;
    a.rows = P.F.rows;
    a.subperm = P.F.subperm;
    // one thread per window row; 32-column sub-steps only for nb <= 128 (trail LDS)
    const int panel_threads = 2 * nb < 64 ? 64 : 2 * nb;
    if (sw == 32 && panel_threads > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rowblock_prep_kernel, dim3(a.nblk, p), dim3(256), 0, s, a);
    hipLaunchKernelGGL(band_window_init_kernel, dim3(p), dim3(256), 0, s, a);
    int buf = 0;
    for (int k = 0; k < a.nblk; ++k) {
        for (int c0 = 0; c0 < nb; c0 += sw) {
            const bool fin = c0 + sw == nb;
            const int total = (fin ? nb : c0) + 3 * nb - (fin ? nb : c0 + sw);
            const dim3 tg((total + kFacWaves - 1) / kFacWaves, p);
            const size_t tl = trail_lds(sw);
#define RF_FAC_LAUNCH(NS_, SW_)                                                                   \
            hipLaunchKernelGGL((band_panel_kernel<SW_, SW_ == 32 ? 256 : 512>), dim3(p),          \
                               dim3(panel_threads), 0, s, a,                                     \
                               k, buf, c0);                                                      \
            hipLaunchKernelGGL((band_trail_kernel<NS_, SW_>), tg, dim3(kFacThreads), tl, s, a, k,  \
                               buf, c0)
            if (sw == 32) {
                if (ns <= 1) { RF_FAC_LAUNCH(1, 32); }
                else if (ns <= 2) { RF_FAC_LAUNCH(2, 32); }
                else if (ns <= 4) { RF_FAC_LAUNCH(4, 32); }
                else { RF_FAC_LAUNCH(8, 32); }
            } else {
                if (ns <= 1) { RF_FAC_LAUNCH(1, 16); }
                else if (ns <= 2) { RF_FAC_LAUNCH(2, 16); }
                else if (ns <= 4) { RF_FAC_LAUNCH(4, 16); }
                else { RF_FAC_LAUNCH(8, 16); }
            }
#undef RF_FAC_LAUNCH
        }
        buf ^= 1;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb == 128)
        hipLaunchKernelGGL(tri_inverse_reg_kernel<128>, dim3(a.nblk, p, 2), dim3(512), 0, s,
                           P.F.tiles, a.nblk);
    else if (nb == 64)
        hipLaunchKernelGGL(tri_inverse_reg_kernel<64>, dim3(a.nblk, p, 2), dim3(256), 0, s,
                           P.F.tiles, a.nblk);
    else if (size_t(nb) * 32 * sizeof(zd) <= size_t(P.max_lds))
        hipLaunchKernelGGL(tri_inverse_kernel<32>, dim3(a.nblk, p, 2), dim3(kThreads),
                           size_t(nb) * 32 * sizeof(zd), s, P.F.tiles, nb, a.nblk);
    else
        hipLaunchKernelGGL(tri_inverse_kernel<16>, dim3(a.nblk, p, 2), dim3(kThreads),
                           size_t(nb) * 16 * sizeof(zd), s, P.F.tiles, nb, a.nblk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the products of the cluster solve (its own tiles only: a batch owner forms them
    // for every disk)
    if (P.F.ftiles && !P.shared_factors) return launch_fused_tiles(P, s);
    return hipSuccess;
}

// Threads per solve workgroup: 512, or 256 for eight complex128 right-hand sides at tile
// 256, where a wave then has the whole register file for its 4 x 8 accumulators (and the
// forward window sits in three nb-row buffers, see the kernel); eight complex64 ones fit
// the registers of 512 threads.
template <int CW, int NB, typename CT>
constexpr int solve_threads() {
    return (NB == 256 && CW == 8 && sizeof(CT) == sizeof(zd)) ? 256 : kSolveThreads;
}

static size_t solve_lds(int nb, int cw, size_t elem, bool inplace) {
    // in place: ring (its first 2nb rows hold the window) + ybuf; otherwise
    // win + win2 (2nb each) + ybuf (nb) + ring (3nb); all x cw
    if (inplace) return size_t(4 * nb * cw) * elem;
    return size_t(2 * nb * cw * 2 + nb * cw + 3 * nb * cw) * elem;
}

template <int CW, int NB, typename CT>
static hipError_t launch_solve_nb(const SolveArgs &a, hipStream_t s, bool adjoint) {
    const int slices = (a.ncols + CW - 1) / CW;
    constexpr int NT = solve_threads<CW, NB, CT>();
    if constexpr (NT == kSolveThreads && CW <= 4) {       // adjoint solves: up to four columns
        if (adjoint) {
            hipLaunchKernelGGL((band_solve_adj_kernel<CW, NB, NT, CT>), dim3(slices * a.p), dim3(NT),
                               solve_lds(NB, CW, sizeof(CT), false), s, a);
            return hipGetLastError();
        }
    } else {
        if (adjoint) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((band_solve_kernel<CW, NB, NT, CT>), dim3(slices * a.p), dim3(NT),
                       solve_lds(NB, CW, sizeof(CT), NT < kSolveThreads), s, a);
    return hipGetLastError();
}

template <int CW, typename CT>
static hipError_t launch_solve_cw(const SolveArgs &a, hipStream_t s, bool adjoint = false) {
    switch (a.nb) {
        case 16: return launch_solve_nb<CW, 16, CT>(a, s, adjoint);
        case 32: return launch_solve_nb<CW, 32, CT>(a, s, adjoint);
        case 64: return launch_solve_nb<CW, 64, CT>(a, s, adjoint);
        case 128: return launch_solve_nb<CW, 128, CT>(a, s, adjoint);
        case 256: return launch_solve_nb<CW, 256, CT>(a, s, adjoint);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tiles_adjoint(const rf_plan &P, const rf_plan &parent, hipStream_t s) {
    const int p = P.opts.p, nblk = P.F.nblk, nb = P.F.nb;
    if (parent.opts.p != p || parent.F.nblk != nblk || parent.F.nb != nb) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tiles_adjoint_kernel, dim3(nblk * 5, p), dim3(256), 0, s, parent.F.tiles,
                       P.F.tiles, p, nblk, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t pb = size_t(nblk) * 2 * nb * sizeof(int32_t);
    for (int i = 0; i < p; ++i) {
        e = hipMemcpyAsync(P.F.perm + int64_t(i) * nblk * 2 * nb,
                           parent.F.perm + int64_t(p - 1 - i) * nblk * 2 * nb, pb,
                           hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
__global__ void to_c64_kernel(const zd *src, zf *dst, int64_t count) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const zd v = src[e];
    dst[e] = fmake(float(v.x), float(v.y));
}
}  // namespace

hipError_t launch_tiles_to_c64(const rf_plan &P, hipStream_t s) {
    if (!P.F.tiles32) return hipErrorInvalidValue;
    const int64_t count = int64_t(P.opts.p) * P.F.nblk * 5 * P.F.tile_elems;
    hipLaunchKernelGGL(to_c64_kernel, dim3((count + 255) / 256), dim3(256), 0, s, P.F.tiles,
                       P.F.tiles32, count);
    return hipGetLastError();
}

namespace {

// complex128 solves of this plan run as clusters over the fused tiles
bool cluster_path(const rf_plan &P) {
    return P.opts.precision == 0 && !P.F.adjoint && P.F.ftiles && P.F.cluster_ok &&
           cluster_solve_supported(P.F.nb);
}

// Work blocks of one application of G to ncols columns: B X staging (only when B is not
// diagonal), per-pole forward results (tile precision) and per-pole weighted solutions.
struct InnerBufs {
    zd *rhs;
    void *ypart;
    zd *xpart;
    zd *refres;          // refinement residuals (plans with refine > 0)
    bool profile;        // record the solve launch in the plan's kernel statistics
};

hipError_t inner_apply_core(const rf_plan &P, const zd *X, int64_t ldx, int ncols, zd *Z,
                            int64_t ldz, hipStream_t s, bool apply_b, const zd *colw,
                            const InnerBufs &buf) {
    SolveArgs a;
    a.n = int(P.n); a.nb = P.F.nb; a.nblk = P.F.nblk; a.p = P.opts.p;
    a.ncols = ncols;
    const bool c64 = P.opts.precision == 1;
    if (c64 && !P.F.tiles32) return hipErrorInvalidValue;
    a.tiles = c64 ? static_cast<const void *>(P.F.tiles32) : static_cast<const void *>(P.F.tiles);
    a.perm = P.F.perm; a.weights = P.d_weights; a.colw = colw;
    a.ypart = buf.ypart; a.xpart = buf.xpart;
    a.npad = int64_t(P.F.nblk) * P.F.nb;
    a.x_pole_stride = 0; a.unit_weight = 0; a.accumulate = 0;
    if (!apply_b) {
        a.X = X; a.ldx = ldx; a.bdiag = nullptr;
    } else if (P.B.diagonal) {
        a.X = X; a.ldx = ldx; a.bdiag = P.B.dval;
    } else {
        hipError_t e = launch_spmm(P.B, ncols, X, ldx, buf.rhs, a.npad, s);
        if (e != hipSuccess) return e;
        a.X = buf.rhs; a.ldx = a.npad; a.bdiag = nullptr;
    }
    const bool adj = P.F.adjoint;
    // eight right-hand sides per workgroup: solves at tile 256 only (not the adjoint's)
    const bool cw8 = !adj && a.nb == 256;
    int cw = P.opts.trsm_cols;
    if (cw <= 0) {
        // the narrowest slices whose workgroups all run at once, one per compute unit
        // (a second workgroup on a unit only queues behind the first's tile stream)
        cw = 1;
        while (cw < (cw8 ? 8 : 4) && (int64_t(ncols + cw - 1) / cw) * a.p > P.num_cu) cw *= 2;
    }
    if (cw > 4) cw = cw8 ? 8 : 4;
    else if (cw > 2) cw = 4;
    const size_t elem = c64 ? sizeof(zf) : sizeof(zd);
    // (the three-buffer window: eight complex128 columns, the 256-thread form)
    while (cw > 1 && solve_lds(a.nb, cw, elem, cw == 8 && !c64) > size_t(P.max_lds)) cw /= 2;
    hipError_t e;
    hipEvent_t ev0 = nullptr;
    if (buf.profile) P.prof.record_begin(s, ev0);
    if (adj && (c64 || colw)) return hipErrorInvalidValue;
    if (cluster_path(P)) {
        // complex128 solves over the fused tiles, a cluster of workgroups per pole and
        // 16 right-hand sides
        e = launch_cluster_solve(P, ClusterSolve{a.X, a.ldx, a.bdiag, buf.rhs, 0, colw,
                                                 static_cast<zd *>(buf.ypart), buf.xpart, ncols,
                                                 0, 0}, s);
        if (e != hipSuccess) return e;
        if (buf.profile) P.prof.record_end(s, ev0, ncols, 0);
        int64_t tot = P.n * ncols;
        hipLaunchKernelGGL(pole_sum_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, buf.xpart,
                           a.p, a.npad, P.n, ncols, Z, ldz);
        return hipGetLastError();
    }
    auto solve = [&](const SolveArgs &sa) -> hipError_t {
        if (c64) {
            switch (cw) {
                case 1: return launch_solve_cw<1, zf>(sa, s);
                case 2: return launch_solve_cw<2, zf>(sa, s);
                case 8: return launch_solve_nb<8, 256, zf>(sa, s, false);   // cw8: tile 256
                default: return launch_solve_cw<4, zf>(sa, s);
            }
        }
        switch (cw) {
            case 1: return launch_solve_cw<1, zd>(sa, s, adj);
            case 2: return launch_solve_cw<2, zd>(sa, s, adj);
            case 8: return launch_solve_nb<8, 256, zd>(sa, s, adj);     // cw8: tile 256
            default: return launch_solve_cw<4, zd>(sa, s, adj);
        }
    };
    e = solve(a);
    if (e != hipSuccess) return e;
    // FP64 iterative refinement of every shifted solve: residual in complex128 from the
    // sparse A and B, correction with the complex64 factors, added to the solution
    const int nref = c64 ? P.opts.refine : 0;
    if (nref > 0 && !buf.refres) return hipErrorInvalidValue;
    for (int it = 0; it < nref; ++it) {
        const int64_t tot = int64_t(P.n) * ncols * a.p;
        hipLaunchKernelGGL(refine_residual_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, int(P.n),
                           ncols, a.p, a.npad, X, ldx, (apply_b && P.B.diagonal) ? P.B.dval : nullptr,
                           (apply_b && !P.B.diagonal) ? buf.rhs : nullptr, P.A.rowptr, P.A.colind,
                           P.A.val, P.B.rowptr, P.B.colind, P.B.val, P.d_poles, P.d_weights, colw,
                           buf.xpart, buf.refres);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        SolveArgs ra = a;
        ra.X = buf.refres; ra.ldx = a.npad; ra.bdiag = nullptr;
        ra.x_pole_stride = a.npad * ncols;
        ra.unit_weight = 1; ra.accumulate = 1;
        e = solve(ra);
        if (e != hipSuccess) return e;
    }
    if (buf.profile) P.prof.record_end(s, ev0, ncols, 0);
    int64_t tot = P.n * ncols;
    hipLaunchKernelGGL(pole_sum_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, buf.xpart, a.p,
                       a.npad, P.n, ncols, Z, ldz);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_inner_apply(const rf_plan &P, const zd *X, int64_t ldx, int ncols, zd *Z,
                              int64_t ldz, hipStream_t s, bool apply_b, const zd *colw) {
    return inner_apply_core(P, X, ldx, ncols, Z, ldz, s, apply_b, colw,
                            InnerBufs{P.rhs, P.ypart, P.xpart, P.refres, true});
}

// ---------------------------------------------------------------------------
// Allocation-free application of G: the work blocks live in one file-scope device
// array instead of plan buffers.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is passed to
// kernels; the array's name in host code is not a device address.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t inner_scratch_capacity() { return kScratchBytes; }

size_t inner_scratch_per_column(const rf_plan &P) {
    const int64_t npad = int64_t(P.F.nblk) * P.F.nb;
    const size_t ye = P.opts.precision == 1 ? sizeof(zf) : sizeof(zd);
    const size_t rhs = (P.B.diagonal && !cluster_path(P)) ? 0 : size_t(npad) * sizeof(zd);
    const size_t ref = P.opts.precision == 1 && P.opts.refine > 0 ? sizeof(zd) : 0;
    return rhs + size_t(P.opts.p) * npad * (ye + sizeof(zd) + ref);
}

hipError_t launch_inner_apply_static(const rf_plan &P, const zd *X, int64_t ldx, int ncols,
                                     zd *Z, int64_t ldz, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            g_scratch_ptr[dev] = ptr;
        }
        base = g_scratch_ptr[dev];
    }
    const int64_t npad = int64_t(P.F.nblk) * P.F.nb;
    const size_t ye = P.opts.precision == 1 ? sizeof(zf) : sizeof(zd);
    // columns per chunk: the largest count whose three blocks (each 256-byte aligned) fit
    int chunk = ncols;
    const bool ref = P.opts.precision == 1 && P.opts.refine > 0;
    const bool staged = !P.B.diagonal || cluster_path(P);   // B X staging block
    auto need = [&](int k) {
        const size_t rhs = staged ? align256(size_t(npad) * k * sizeof(zd)) : 0;
        return rhs + align256(size_t(P.opts.p) * npad * k * ye) +
               align256(size_t(P.opts.p) * npad * k * sizeof(zd)) +
               (ref ? align256(size_t(P.opts.p) * npad * k * sizeof(zd)) : 0);
    };
    while (chunk > 0 && need(chunk) > kScratchBytes) --chunk;
    if (chunk == 0) return hipErrorInvalidValue;          // one column does not fit
    unsigned char *b = static_cast<unsigned char *>(base);
    for (int c0 = 0; c0 < ncols; c0 += chunk) {
        const int k = std::min(chunk, ncols - c0);
        InnerBufs buf;
        size_t off = 0;
        buf.rhs = nullptr;
        if (staged) {
            buf.rhs = reinterpret_cast<zd *>(b + off);
            off += align256(size_t(npad) * k * sizeof(zd));
        }
        buf.ypart = b + off;
        off += align256(size_t(P.opts.p) * npad * k * ye);
        buf.xpart = reinterpret_cast<zd *>(b + off);
        off += align256(size_t(P.opts.p) * npad * k * sizeof(zd));
        buf.refres = ref ? reinterpret_cast<zd *>(b + off) : nullptr;
        buf.profile = false;
        e = inner_apply_core(P, X + int64_t(c0) * ldx, ldx, k, Z + int64_t(c0) * ldz, ldz, s, true,
                             nullptr, buf);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
