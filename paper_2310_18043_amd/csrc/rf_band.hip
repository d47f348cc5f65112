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
    zd *window;         // [pole][2nb x 3nb], ld 2nb
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

// One workgroup factors one pole.  NC = columns per in-LDS chunk of the panel.
template <int NC>
__global__ __launch_bounds__(kThreads) void band_factor_kernel(FactorArgs a) {
    const int pole = blockIdx.x;
    const int nb = a.nb, nblk = a.nblk;
    const int ldw = 2 * nb;
    const int64_t te = int64_t(nb) * nb;
    zd *W = a.window + int64_t(pole) * (2 * nb) * (3 * nb);
    const zd z = a.poles[pole];
    const int tid = threadIdx.x;

    extern __shared__ unsigned char smem_raw[];
    zd *C = reinterpret_cast<zd *>(smem_raw);                    // [2nb][NC], row-major
    int *pivrow = reinterpret_cast<int *>(C + 2 * nb * NC);      // [nb]
    double *redv = reinterpret_cast<double *>(pivrow + nb);      // [kThreads/64]
    int *redi = reinterpret_cast<int *>(redv + kThreads / 64);   // [kThreads/64]
    __shared__ int s_info;

    if (tid == 0) s_info = 0;
    // window for k = 0
    for (int64_t e = tid; e < int64_t(2 * nb) * (3 * nb); e += kThreads) W[e] = zmake(0, 0);
    __syncthreads();
    scatter_rows(a, z, W, ldw, 0, 0, 0);
    if (nblk > 1) scatter_rows(a, z, W, ldw, 1, 1, 0);
    __syncthreads();

    for (int k = 0; k < nblk; ++k) {
        const int rows = (k + 1 < nblk) ? 2 * nb : nb;
        const int cols = min(3 * nb, (nblk - k) * nb);
        for (int jc = 0; jc < nb; jc += NC) {
            // ---- load chunk (rows x NC) into LDS
            for (int e = tid; e < rows * NC; e += kThreads) {
                int r = e % rows, cc = e / rows;
                C[r * NC + cc] = W[r + int64_t(jc + cc) * ldw];
            }
            __syncthreads();
            // ---- unblocked LU with partial pivoting on the chunk
            for (int cc = 0; cc < NC; ++cc) {
                const int j = jc + cc;
                double best = -1.0; int bi = j;
                for (int r = j + tid; r < rows; r += kThreads) {
                    double v = zabs2(C[r * NC + cc]);
                    if (v > best) { best = v; bi = r; }
                }
                // wave reduction (first index wins ties)
                for (int off = 32; off > 0; off >>= 1) {
                    double ov = __shfl_down(best, off, 64);
                    int oi = __shfl_down(bi, off, 64);
                    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
                }
                if ((tid & 63) == 0) { redv[tid >> 6] = best; redi[tid >> 6] = bi; }
                __syncthreads();
                if (tid == 0) {
                    double bv = redv[0]; int bidx = redi[0];
                    for (int wv = 1; wv < kThreads / 64; ++wv)
                        if (redv[wv] > bv || (redv[wv] == bv && redi[wv] < bidx)) {
                            bv = redv[wv]; bidx = redi[wv];
                        }
                    if (!(bv > 0.0)) {            // exact zero (or NaN) pivot
                        if (s_info == 0) s_info = k * nb + j + 1;
                        bidx = j;
                    }
                    pivrow[j] = bidx;
                }
                __syncthreads();
                const int pr = pivrow[j];
                if (pr != j && tid < NC) {
                    zd t = C[j * NC + tid]; C[j * NC + tid] = C[pr * NC + tid]; C[pr * NC + tid] = t;
                }
                __syncthreads();
                const zd piv = C[j * NC + cc];
                const bool zero = !(zabs2(piv) > 0.0);
                const zd inv = zero ? zmake(0, 0) : zdiv(zmake(1.0, 0.0), piv);
                for (int r = j + 1 + tid; r < rows; r += kThreads) {
                    zd l = zmul(C[r * NC + cc], inv);
                    C[r * NC + cc] = l;
                    for (int c2 = cc + 1; c2 < NC; ++c2) zfms(C[r * NC + c2], l, C[j * NC + c2]);
                }
                __syncthreads();
            }
            // ---- write chunk back
            for (int e = tid; e < rows * NC; e += kThreads) {
                int r = e % rows, cc = e / rows;
                W[r + int64_t(jc + cc) * ldw] = C[r * NC + cc];
            }
            // ---- apply the chunk's interchanges to the other window columns
            for (int col = tid; col < cols; col += kThreads) {
                if (col >= jc && col < jc + NC) continue;
                zd *wc = W + int64_t(col) * ldw;
                for (int cc = 0; cc < NC; ++cc) {
                    int j = jc + cc, pr = pivrow[j];
                    if (pr != j) { zd t = wc[j]; wc[j] = wc[pr]; wc[pr] = t; }
                }
            }
            __syncthreads();
            // ---- U12 = L_chunk^{-1} W[chunk rows, right columns]
            for (int col = jc + NC + tid; col < cols; col += kThreads) {
                zd *wc = W + int64_t(col) * ldw;
                zd u[NC];
                for (int cc = 0; cc < NC; ++cc) {
                    zd v = wc[jc + cc];
                    for (int c2 = 0; c2 < cc; ++c2) zfms(v, C[(jc + cc) * NC + c2], u[c2]);
                    u[cc] = v;
                    wc[jc + cc] = v;
                }
            }
            __syncthreads();
            // ---- trailing update of rows below the chunk, columns right of it
            {
                const int r0 = jc + NC;
                for (int r = r0 + tid; r < rows; r += kThreads) {
                    zd l[NC];
                    for (int cc = 0; cc < NC; ++cc) l[cc] = C[r * NC + cc];
                    for (int col = jc + NC; col < cols; ++col) {
                        const zd *wc = W + int64_t(col) * ldw;
                        zd acc = wc[r];
                        for (int cc = 0; cc < NC; ++cc) zfms(acc, l[cc], wc[jc + cc]);
                        W[r + int64_t(col) * ldw] = acc;
                    }
                }
            }
            __syncthreads();
        }
        // ---- permutation of the window rows: new row i = old row perm[i]
        int32_t *pm = a.perm + (int64_t(pole) * nblk + k) * (2 * nb);
        if (tid == 0) {
            for (int i = 0; i < 2 * nb; ++i) pm[i] = i;
            for (int j = 0; j < nb; ++j) {
                int pr = pivrow[j];
                int t = pm[j]; pm[j] = pm[pr]; pm[pr] = t;
            }
        }
        // ---- tiles: L21, U1, U2 straight copies
        zd *T0 = a.tiles + tile_index(pole, k, 0, nblk, te);   // Linv
        zd *T1 = T0 + te;                                      // L21
        zd *T2 = T1 + te;                                      // Uinv
        zd *T3 = T2 + te;                                      // U1
        zd *T4 = T3 + te;                                      // U2
        for (int64_t e = tid; e < te; e += kThreads) {
            int r = int(e % nb), c = int(e / nb);
            T1[e] = (k + 1 < nblk) ? W[nb + r + int64_t(c) * ldw] : zmake(0, 0);
            T3[e] = W[r + int64_t(nb + c) * ldw];
            T4[e] = W[r + int64_t(2 * nb + c) * ldw];
        }
        // diagonal block (packed L11 \ U11) goes to both Linv and Uinv slots; the
        // triangles are inverted in place afterwards by tri_inverse_kernel
        for (int64_t e = tid; e < te; e += kThreads) {
            int r = int(e % nb), c = int(e / nb);
            zd v = W[r + int64_t(c) * ldw];
            T0[e] = v;
            T2[e] = v;
        }
        __syncthreads();
        // ---- slide the window: rows of block k+1 (cols k+1, k+2) move to the top
        if (k + 1 < nblk) {
            for (int64_t e = tid; e < int64_t(nb) * (2 * nb); e += kThreads) {
                int r = int(e % nb), c = int(e / nb);
                W[r + int64_t(c) * ldw] = W[nb + r + int64_t(nb + c) * ldw];
            }
            __syncthreads();
            for (int64_t e = tid; e < int64_t(2 * nb) * (3 * nb); e += kThreads) {
                int r = int(e % (2 * nb)), c = int(e / (2 * nb));
                if (r >= nb || c >= 2 * nb) W[e] = zmake(0, 0);
            }
            __syncthreads();
            if (k + 2 < nblk) scatter_rows(a, z, W, ldw, 1, k + 2, (k + 1) * nb);
            __syncthreads();
        }
    }
    if (tid == 0) a.info[pole] = s_info;
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

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
struct SolveArgs {
    int n, nb, nblk, p;
    int ncols;               // total right-hand sides
    const zd *X; int64_t ldx;        // right-hand sides (before B)
    const zd *bdiag;                 // diagonal of B, or null (then X already holds B X)
    const zd *tiles;
    const int32_t *perm;
    const zd *weights;
    zd *ypart;               // [pole][npad x ncols]  forward results
    zd *xpart;               // [pole][npad x ncols]  w_i * K_i^{-1} B X
    int64_t npad;
};

// Partial products of T (nb x nb, global, column-major) times v (LDS, [nb][CW]).
// G = floor(256/nb) threads share an output row i, each summing a contiguous
// range of the inner index; partial sums go to red[(g*nb + i)*CW + c] and are
// added by tile_reduce after a barrier.  Threads with g >= G idle.
template <int CW>
__device__ inline void tile_gemv(const zd *__restrict__ T, const zd *v, zd *red, int nb) {
    const int tid = threadIdx.x;
    const int G = kThreads / nb;         // threads per output row (>= 1, nb <= 256)
    const int i = tid % nb, g = tid / nb;
    if (g >= G) return;
    const int klen = (nb + G - 1) / G;
    const int k0 = g * klen;
    const int k1 = min(nb, k0 + klen);
    zd acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = zmake(0, 0);
    const zd *tp = T + i;
    for (int kk = k0; kk < k1; ++kk) {
        zd t = tp[int64_t(kk) * nb];
        const zd *vr = v + kk * CW;
#pragma unroll
        for (int c = 0; c < CW; ++c) zfma(acc[c], t, vr[c]);
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) red[(g * nb + i) * CW + c] = acc[c];
}

// sum the G partial products of row i (called after a barrier); returns via out
template <int CW>
__device__ inline void tile_reduce(const zd *red, int nb, int i, zd *out) {
    const int G = kThreads / nb;
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        zd s = red[i * CW + c];
        for (int g = 1; g < G; ++g) s = zadd(s, red[(g * nb + i) * CW + c]);
        out[c] = s;
    }
}

template <int CW>
__global__ __launch_bounds__(kThreads) void band_solve_kernel(SolveArgs a) {
    const int p = a.p;
    const int pole = blockIdx.x % p;             // slices of one pole share an XCD
    const int slice = blockIdx.x / p;
    const int c0 = slice * CW;
    if (c0 >= a.ncols) return;
    const int ncw = min(CW, a.ncols - c0);
    const int nb = a.nb, nblk = a.nblk;
    const int64_t te = int64_t(nb) * nb;
    const int tid = threadIdx.x;
    const zd wgt = a.weights[pole];

    extern __shared__ unsigned char smem_raw[];
    zd *win = reinterpret_cast<zd *>(smem_raw);   // [2nb][CW]
    zd *win2 = win + 2 * nb * CW;                 // [2nb][CW]
    zd *ybuf = win2 + 2 * nb * CW;                // [nb][CW]
    zd *ring = ybuf + nb * CW;                    // [3][nb][CW]
    zd *red = ring + 3 * nb * CW;                 // [kThreads][CW]

    zd *yp = a.ypart + int64_t(pole) * a.npad * a.ncols;
    zd *xp = a.xpart + int64_t(pole) * a.npad * a.ncols;
    const zd *tiles = a.tiles + int64_t(pole) * nblk * 5 * te;
    const int32_t *perm = a.perm + int64_t(pole) * nblk * 2 * nb;

    auto load_rhs = [&](int blk, zd *dst) {
        for (int e = tid; e < nb * CW; e += kThreads) {
            int r = e / CW, c = e % CW;
            int64_t row = int64_t(blk) * nb + r;
            zd v = zmake(0, 0);
            if (row < a.n && c < ncw) {
                v = a.X[row + int64_t(c0 + c) * a.ldx];
                if (a.bdiag) v = zmul(a.bdiag[row], v);
            }
            dst[r * CW + c] = v;
        }
    };

    // ---------------- forward sweep
    load_rhs(0, win);
    for (int k = 0; k < nblk; ++k) {
        const bool last = (k + 1 == nblk);
        if (!last) load_rhs(k + 1, win + nb * CW);
        __syncthreads();
        const int rows = last ? nb : 2 * nb;
        const int32_t *pk = perm + int64_t(k) * 2 * nb;
        for (int e = tid; e < rows * CW; e += kThreads) {
            int r = e / CW, c = e % CW;
            win2[e] = win[pk[r] * CW + c];
        }
        __syncthreads();
        const zd *Tk = tiles + int64_t(k) * 5 * te;
        tile_gemv<CW>(Tk, win2, red, nb);            // Linv * w_top
        __syncthreads();
        if (tid < nb) {
            zd o[CW];
            tile_reduce<CW>(red, nb, tid, o);
#pragma unroll
            for (int c = 0; c < CW; ++c) ybuf[tid * CW + c] = o[c];
        }
        __syncthreads();
        for (int e = tid; e < nb * CW; e += kThreads) {
            int r = e / CW, c = e % CW;
            if (c < ncw) yp[int64_t(k) * nb + r + int64_t(c0 + c) * a.npad] = ybuf[e];
        }
        if (!last) {
            tile_gemv<CW>(Tk + te, ybuf, red, nb);   // L21 * y_k
            __syncthreads();
            if (tid < nb) {
                zd o[CW];
                tile_reduce<CW>(red, nb, tid, o);
#pragma unroll
                for (int c = 0; c < CW; ++c)
                    win[tid * CW + c] = zsub(win2[(nb + tid) * CW + c], o[c]);
            }
        }
        __syncthreads();
    }
    __threadfence_block();
    // ---------------- backward sweep
    for (int e = tid; e < 3 * nb * CW; e += kThreads) ring[e] = zmake(0, 0);
    __syncthreads();
    for (int k = nblk - 1; k >= 0; --k) {
        zd *xk = ring + (k % 3) * nb * CW;
        const zd *xk1 = ring + ((k + 1) % 3) * nb * CW;
        const zd *xk2 = ring + ((k + 2) % 3) * nb * CW;
        const zd *Tk = tiles + int64_t(k) * 5 * te;
        // v = y_k - U1 x_{k+1} - U2 x_{k+2}, accumulated in ybuf
        for (int e = tid; e < nb * CW; e += kThreads) {
            int r = e / CW, c = e % CW;
            ybuf[e] = (c < ncw) ? yp[int64_t(k) * nb + r + int64_t(c0 + c) * a.npad] : zmake(0, 0);
        }
        __syncthreads();
        if (k + 1 < nblk) {
            tile_gemv<CW>(Tk + 3 * te, xk1, red, nb);
            __syncthreads();
            if (tid < nb) {
                zd o[CW];
                tile_reduce<CW>(red, nb, tid, o);
#pragma unroll
                for (int c = 0; c < CW; ++c) ybuf[tid * CW + c] = zsub(ybuf[tid * CW + c], o[c]);
            }
            __syncthreads();
        }
        if (k + 2 < nblk) {
            tile_gemv<CW>(Tk + 4 * te, xk2, red, nb);
            __syncthreads();
            if (tid < nb) {
                zd o[CW];
                tile_reduce<CW>(red, nb, tid, o);
#pragma unroll
                for (int c = 0; c < CW; ++c) ybuf[tid * CW + c] = zsub(ybuf[tid * CW + c], o[c]);
            }
            __syncthreads();
        }
        tile_gemv<CW>(Tk + 2 * te, ybuf, red, nb);   // Uinv * v
        __syncthreads();
        if (tid < nb) {
            zd o[CW];
            tile_reduce<CW>(red, nb, tid, o);
#pragma unroll
            for (int c = 0; c < CW; ++c) xk[tid * CW + c] = o[c];
        }
        __syncthreads();
        for (int e = tid; e < nb * CW; e += kThreads) {
            int r = e / CW, c = e % CW;
            if (c < ncw) xp[int64_t(k) * nb + r + int64_t(c0 + c) * a.npad] = zmul(wgt, xk[e]);
        }
        __syncthreads();
    }
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
    auto factor_lds = [&](int nc) {
        return size_t(2 * nb * nc) * sizeof(zd) + nb * sizeof(int) +
               (kThreads / 64) * (sizeof(double) + sizeof(int));
    };
    if (factor_lds(16) <= size_t(P.max_lds)) {
        hipLaunchKernelGGL(band_factor_kernel<16>, dim3(p), dim3(kThreads), factor_lds(16), s, a);
    } else if (factor_lds(8) <= size_t(P.max_lds)) {
        hipLaunchKernelGGL(band_factor_kernel<8>, dim3(p), dim3(kThreads), factor_lds(8), s, a);
    } else {
        hipLaunchKernelGGL(band_factor_kernel<4>, dim3(p), dim3(kThreads), factor_lds(4), s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (size_t(nb) * 32 * sizeof(zd) <= size_t(P.max_lds))
        hipLaunchKernelGGL(tri_inverse_kernel<32>, dim3(a.nblk, p, 2), dim3(kThreads),
                           size_t(nb) * 32 * sizeof(zd), s, P.F.tiles, nb, a.nblk);
    else
        hipLaunchKernelGGL(tri_inverse_kernel<16>, dim3(a.nblk, p, 2), dim3(kThreads),
                           size_t(nb) * 16 * sizeof(zd), s, P.F.tiles, nb, a.nblk);
    return hipGetLastError();
}

static size_t solve_lds(int nb, int cw) {
    // win + win2 (2nb each) + ybuf (nb) + ring (3nb) + red (kThreads), all x cw
    return size_t(2 * nb * cw * 2 + nb * cw + 3 * nb * cw + kThreads * cw) * sizeof(zd);
}

template <int CW>
static hipError_t launch_solve_cw(const SolveArgs &a, hipStream_t s) {
    const int slices = (a.ncols + CW - 1) / CW;
    hipLaunchKernelGGL(band_solve_kernel<CW>, dim3(slices * a.p), dim3(kThreads),
                       solve_lds(a.nb, CW), s, a);
    return hipGetLastError();
}

hipError_t launch_inner_apply(const rf_plan &P, const zd *X, int64_t ldx, int ncols, zd *Z,
                              int64_t ldz, hipStream_t s) {
    SolveArgs a;
    a.n = int(P.n); a.nb = P.F.nb; a.nblk = P.F.nblk; a.p = P.opts.p;
    a.ncols = ncols;
    a.tiles = P.F.tiles; a.perm = P.F.perm; a.weights = P.d_weights;
    a.ypart = P.ypart; a.xpart = P.xpart;
    a.npad = int64_t(P.F.nblk) * P.F.nb;
    if (P.B.diagonal) {
        a.X = X; a.ldx = ldx; a.bdiag = P.B.dval;
    } else {
        hipError_t e = launch_spmm(P.B, ncols, X, ldx, P.rhs, a.npad, s);
        if (e != hipSuccess) return e;
        a.X = P.rhs; a.ldx = a.npad; a.bdiag = nullptr;
    }
    int cw = P.opts.trsm_cols;
    if (cw <= 0) {
        // enough workgroups to cover the chip, at most 8 columns each
        cw = 8;
        while (cw > 1 && (int64_t(ncols + cw - 1) / cw) * a.p < 256) cw /= 2;
    }
    if (cw > 4) cw = 8; else if (cw > 2) cw = 4;
    while (cw > 1 && solve_lds(a.nb, cw) > size_t(P.max_lds)) cw /= 2;
    hipError_t e;
    switch (cw) {
        case 1: e = launch_solve_cw<1>(a, s); break;
        case 2: e = launch_solve_cw<2>(a, s); break;
        case 4: e = launch_solve_cw<4>(a, s); break;
        default: e = launch_solve_cw<8>(a, s); break;
    }
    if (e != hipSuccess) return e;
    int64_t tot = P.n * ncols;
    hipLaunchKernelGGL(pole_sum_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, P.xpart, a.p,
                       a.npad, P.n, ncols, Z, ldz);
    return hipGetLastError();
}
