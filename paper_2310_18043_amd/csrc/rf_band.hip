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

// The factorization runs as a sequence of launches per block step k, all p poles
// at once:
//   band_panel_kernel  (one workgroup per pole): LU with partial pivoting of the
//       2nb x nb panel (column block k of the window), chunk by chunk in LDS;
//       stores the row permutation, the packed L11 \ U11 block and L21;
//   band_update_kernel (2nb/CPW workgroups per pole, CPW columns each): applies
//       the permutation to the U part of the window (column blocks k+1, k+2),
//       U_top = L11^{-1} (top rows) by blocked substitution in LDS, bottom rows
//       minus L21 U_top, stores U1/U2 and writes the updated bottom rows into the
//       next window; workgroup 0 of each pole also loads the next row block.
// Kernel boundaries order the steps, so no workgroup ever waits on another.
// The window of each pole is double-buffered (current / next).

__device__ inline zd *pole_window(zd *base, int pole, int buf, int nb) {
    return base + (int64_t(pole) * 2 + buf) * (2 * nb) * (3 * nb);
}

// zero window rows [h*nb, h*nb+nb) and load row block rb of K = z B - A into them
__device__ void load_row_block(const FactorArgs &a, zd z, zd *W, int h, int rb, int cbase) {
    const int nb = a.nb, ldw = 2 * nb;
    for (int e = threadIdx.x; e < nb * 3 * nb; e += blockDim.x) {
        int r = e % nb, c = e / nb;
        W[h * nb + r + int64_t(c) * ldw] = zmake(0, 0);
    }
    __syncthreads();
    scatter_rows(a, z, W, ldw, h, rb, cbase);
    __syncthreads();
}

__global__ __launch_bounds__(256) void band_window_init_kernel(FactorArgs a) {
    const int pole = blockIdx.x;
    zd *W = pole_window(a.window, pole, 0, a.nb);
    const zd z = a.poles[pole];
    load_row_block(a, z, W, 0, 0, 0);
    if (a.nblk > 1) load_row_block(a, z, W, 1, 1, 0);
    else {
        for (int e = threadIdx.x; e < a.nb * 3 * a.nb; e += blockDim.x) {
            int r = e % a.nb, c = e / a.nb;
            W[a.nb + r + int64_t(c) * 2 * a.nb] = zmake(0, 0);
        }
    }
    if (threadIdx.x == 0) a.info[pole] = 0;
}

template <int NC>
__global__ __launch_bounds__(kThreads) void band_panel_kernel(FactorArgs a, int k, int buf) {
    const int pole = blockIdx.x;
    const int nb = a.nb, nblk = a.nblk;
    const int ldw = 2 * nb;
    const int64_t te = int64_t(nb) * nb;
    zd *W = pole_window(a.window, pole, buf, nb);
    const int tid = threadIdx.x;
    extern __shared__ unsigned char smem_raw[];
    zd *C = reinterpret_cast<zd *>(smem_raw);                    // [2nb][NC], row-major
    zd *U12 = C + 2 * nb * NC;                                   // [NC][nb]
    int *pivrow = reinterpret_cast<int *>(U12 + NC * nb);        // [nb]
    int *srcrow = pivrow + nb;                                   // [2 NC]
    int *dstrow = srcrow + 2 * NC;                               // [2 NC]
    double *redv = reinterpret_cast<double *>(dstrow + 2 * NC);  // [kThreads/64]
    int *redi = reinterpret_cast<int *>(redv + kThreads / 64);   // [kThreads/64]
    __shared__ int s_info, s_nmoved;
    if (tid == 0) s_info = 0;
    const int rows = (k + 1 < nblk) ? 2 * nb : nb;
    for (int jc = 0; jc < nb; jc += NC) {
        for (int e = tid; e < rows * NC; e += kThreads) {
            int r = e % rows, cc = e / rows;
            C[r * NC + cc] = W[r + int64_t(jc + cc) * ldw];
        }
        __syncthreads();
        // ---- unblocked LU with partial pivoting of the chunk, in LDS
        for (int cc = 0; cc < NC; ++cc) {
            const int j = jc + cc;
            double best = -1.0; int bi = j;
            for (int r = j + tid; r < rows; r += kThreads) {
                double v = zabs2(C[r * NC + cc]);
                if (v > best) { best = v; bi = r; }
            }
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
                    if (redv[wv] > bv || (redv[wv] == bv && redi[wv] < bidx)) { bv = redv[wv]; bidx = redi[wv]; }
                if (!(bv > 0.0)) { if (s_info == 0) s_info = k * nb + j + 1; bidx = j; }
                pivrow[j] = bidx;
            }
            __syncthreads();
            const int pr = pivrow[j];
            if (pr != j && tid < NC) {
                zd t = C[j * NC + tid]; C[j * NC + tid] = C[pr * NC + tid]; C[pr * NC + tid] = t;
            }
            __syncthreads();
            const zd piv = C[j * NC + cc];
            const zd inv = (zabs2(piv) > 0.0) ? zdiv(zmake(1.0, 0.0), piv) : zmake(0, 0);
            for (int r = j + 1 + tid; r < rows; r += kThreads) {
                zd l = zmul(C[r * NC + cc], inv);
                C[r * NC + cc] = l;
#pragma unroll
                for (int c2 = 0; c2 < NC; ++c2)
                    if (c2 > cc) zfms(C[r * NC + c2], l, C[j * NC + c2]);
            }
            __syncthreads();
        }
        // ---- the chunk's interchanges as one permutation of at most 2 NC rows
        if (tid == 0) {
            int m = 0;
            for (int cc = 0; cc < NC; ++cc) {
                int j = jc + cc, pr = pivrow[j];
                bool hj = false, hp = false;
                for (int q = 0; q < m; ++q) { hj |= (dstrow[q] == j); hp |= (dstrow[q] == pr); }
                if (!hj) { dstrow[m] = j; srcrow[m] = j; ++m; }
                if (!hp && pr != j) { dstrow[m] = pr; srcrow[m] = pr; ++m; }
                // swap the contents (sources) held by rows j and pr
                int qj = -1, qp = -1;
                for (int q = 0; q < m; ++q) { if (dstrow[q] == j) qj = q; if (dstrow[q] == pr) qp = q; }
                if (qj >= 0 && qp >= 0) { int t = srcrow[qj]; srcrow[qj] = srcrow[qp]; srcrow[qp] = t; }
            }
            s_nmoved = m;
        }
        // ---- write the chunk back
        for (int e = tid; e < rows * NC; e += kThreads) {
            int r = e % rows, cc = e / rows;
            W[r + int64_t(jc + cc) * ldw] = C[r * NC + cc];
        }
        __syncthreads();
        // ---- apply the permutation to the other panel columns (independent loads)
        {
            const int m = s_nmoved;
            for (int col = tid; col < nb; col += kThreads) {
                if (col >= jc && col < jc + NC) continue;
                zd *wc = W + int64_t(col) * ldw;
                zd vals[2 * NC];
#pragma unroll
                for (int q = 0; q < 2 * NC; ++q) vals[q] = (q < m) ? wc[srcrow[q]] : zmake(0, 0);
#pragma unroll
                for (int q = 0; q < 2 * NC; ++q) if (q < m) wc[dstrow[q]] = vals[q];
            }
        }
        __syncthreads();
        // ---- U12 inside the panel: one column per thread, values loaded at once
        for (int col = jc + NC + tid; col < nb; col += kThreads) {
            zd *wc = W + int64_t(col) * ldw;
            zd u[NC];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) u[cc] = wc[jc + cc];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
#pragma unroll
                for (int c2 = 0; c2 < NC; ++c2)
                    if (c2 < cc) zfms(u[cc], C[(jc + cc) * NC + c2], u[c2]);
            }
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) { wc[jc + cc] = u[cc]; U12[cc * nb + col] = u[cc]; }
        }
        __syncthreads();
        // ---- trailing update inside the panel (multipliers and U12 from LDS)
        {
            const int r0 = jc + NC, c0 = jc + NC;
            const int nr = rows - r0, ncl = nb - c0;
            const int tot = nr * ncl;
            for (int e0 = tid; e0 < tot; e0 += 4 * kThreads) {
                zd acc[4];
                int rr[4], cl[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int e = e0 + q * kThreads;
                    rr[q] = r0 + (e < tot ? e % nr : 0);
                    cl[q] = c0 + (e < tot ? e / nr : 0);
                    acc[q] = (e < tot) ? W[rr[q] + int64_t(cl[q]) * ldw] : zmake(0, 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int e = e0 + q * kThreads;
                    if (e < tot) {
#pragma unroll
                        for (int cc = 0; cc < NC; ++cc) zfms(acc[q], C[rr[q] * NC + cc], U12[cc * nb + cl[q]]);
                        W[rr[q] + int64_t(cl[q]) * ldw] = acc[q];
                    }
                }
            }
        }
        __syncthreads();
    }
    // permutation of the window rows: new row i = old row perm[i]
    int32_t *pm = a.perm + (int64_t(pole) * nblk + k) * (2 * nb);
    if (tid == 0) {
        for (int i = 0; i < 2 * nb; ++i) pm[i] = i;
        for (int j = 0; j < nb; ++j) {
            int pr = pivrow[j];
            int t = pm[j]; pm[j] = pm[pr]; pm[pr] = t;
        }
        if (s_info != 0 && a.info[pole] == 0) a.info[pole] = s_info;
    }
    // packed L11 \ U11 to both diagonal slots (inverted later), L21
    zd *T0 = a.tiles + tile_index(pole, k, 0, nblk, te);
    zd *T1 = T0 + te, *T2 = T1 + te;
    for (int64_t e = tid; e < te; e += kThreads) {
        int r = int(e % nb), c = int(e / nb);
        zd v = W[r + int64_t(c) * ldw];
        T0[e] = v;
        T2[e] = v;
        T1[e] = (k + 1 < nblk) ? W[nb + r + int64_t(c) * ldw] : zmake(0, 0);
    }
}

// CPW columns of the U part per workgroup.  grid: (2nb/CPW, p)
template <int CPW>
__global__ __launch_bounds__(kThreads) void band_update_kernel(FactorArgs a, int k, int buf) {
    const int pole = blockIdx.y, rank = blockIdx.x;
    const int nb = a.nb, nblk = a.nblk, ldw = 2 * nb;
    const int64_t te = int64_t(nb) * nb;
    const zd *W = pole_window(a.window, pole, buf, nb);
    zd *Wn = pole_window(a.window, pole, buf ^ 1, nb);
    const int tid = threadIdx.x;
    const int rows = (k + 1 < nblk) ? 2 * nb : nb;
    const int cols = min(3 * nb, (nblk - k) * nb);          // window columns that exist
    const int32_t *pm = a.perm + (int64_t(pole) * nblk + k) * (2 * nb);
    zd *T3 = a.tiles + tile_index(pole, k, 3, nblk, te);   // U1
    zd *T4 = T3 + te;                                      // U2
    extern __shared__ unsigned char smem_raw[];
    zd *S = reinterpret_cast<zd *>(smem_raw);              // [2nb][CPW]
    const int cbeg = nb + rank * CPW;                      // first window column of this WG
    // 1. permuted columns into LDS (zeros for columns beyond the matrix)
    for (int e = tid; e < rows * CPW; e += kThreads) {
        int r = e / CPW, c = e % CPW;
        int col = cbeg + c;
        S[e] = (col < cols) ? W[pm[r] + int64_t(col) * ldw] : zmake(0, 0);
    }
    __syncthreads();
    // 2. top rows: U = L11^{-1} S_top, blocks of 16 rows (unit lower L11 from the window)
    zd *Lb = S + 2 * nb * CPW;                             // [2nb][16] L column block
    for (int r0 = 0; r0 < nb; r0 += 16) {
        // stage the 16 multiplier columns r0..r0+15 (rows r0..rows) in LDS
        for (int e = tid; e < (rows - r0) * 16; e += kThreads) {
            int r = r0 + e % (rows - r0), q = e / (rows - r0);
            Lb[r * 16 + q] = W[r + int64_t(r0 + q) * ldw];
        }
        __syncthreads();
        // solve the 16 x 16 unit lower diagonal block: one thread per column
        if (tid < CPW) {
            const int c = tid;
            for (int r = r0 + 1; r < r0 + 16; ++r) {
                zd v = S[r * CPW + c];
                for (int q = r0; q < r; ++q) zfms(v, Lb[r * 16 + (q - r0)], S[q * CPW + c]);
                S[r * CPW + c] = v;
            }
        }
        __syncthreads();
        // rows below the block (all rows of the window, top and bottom): minus L(:, block) U(block)
        for (int e = tid; e < (rows - r0 - 16) * CPW; e += kThreads) {
            int r = r0 + 16 + e / CPW, c = e % CPW;
            zd v = S[r * CPW + c];
#pragma unroll
            for (int q = 0; q < 16; ++q) zfms(v, Lb[r * 16 + q], S[(r0 + q) * CPW + c]);
            S[r * CPW + c] = v;
        }
        __syncthreads();
    }
    // 3. store U1/U2 (top rows) and the updated bottom rows into the next window
    for (int e = tid; e < nb * CPW; e += kThreads) {
        int r = e % nb, c = e / nb;
        int col = cbeg + c;
        if (col < 2 * nb) T3[r + int64_t(col - nb) * nb] = S[r * CPW + c];
        else T4[r + int64_t(col - 2 * nb) * nb] = S[r * CPW + c];
        if (k + 1 < nblk) Wn[r + int64_t(col - nb) * ldw] = S[(nb + r) * CPW + c];
    }
    // 4. workgroup 0: clear the last column block of the next window's top half and
    //    load the fresh row block k+2 into its bottom half
    if (rank == 0 && k + 1 < nblk) {
        for (int e = tid; e < nb * nb; e += kThreads) {
            int r = e % nb, c = e / nb;
            Wn[r + int64_t(2 * nb + c) * ldw] = zmake(0, 0);
        }
        __syncthreads();
        if (k + 2 < nblk) load_row_block(a, a.poles[pole], Wn, 1, k + 2, (k + 1) * nb);
        else {
            for (int e = tid; e < nb * 3 * nb; e += kThreads) {
                int r = e % nb, c = e / nb;
                Wn[nb + r + int64_t(c) * ldw] = zmake(0, 0);
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

// Solve kernel.  One workgroup of NT threads owns one pole and a slice of CW
// right-hand sides and runs the whole forward and backward sweep.  Each nb x nb
// tile product out = T v is done by G threads per output row (G a power of two,
// the G threads of a row sit in adjacent lanes of one wave): thread (i, g) loads
// its contiguous segment of row i of T -- its loads of a tile are issued in
// batches of kSeg, so a tile costs few memory latencies -- multiplies by the
// matching rows of v (LDS, [nb][CW]) and the G partial sums are combined with
// cross-lane shuffles.  Triangular tiles (Linv lower, Uinv upper, U2 lower) are
// read only inside their triangle.  Tiles are read straight from global memory:
// the column slices of one pole run on the same XCD (workgroup id modulo p
// selects the pole) and share each tile through its L2.
constexpr int kSeg = 16;             // tile loads in flight per thread and batch

enum TileShape { kFull = 0, kLower = 1, kUpper = 2 };

struct SolveGeom {
    int G, rows_per_wave, klen;
};

__host__ __device__ inline SolveGeom solve_geom(int nb, int nthreads) {
    SolveGeom g;
    int G = 1;
    while (G * 2 <= 64 && G * 2 * nb <= nthreads) G *= 2;
    g.G = G;
    g.rows_per_wave = 64 / G;
    g.klen = (nb + G - 1) / G;
    return g;
}

// acc[c] = sum_k T[i, k] v[k, c] over this thread's k-segment (clipped to the
// tile's triangle), reduced over the G lanes of row i; valid in lane g == 0.
// Threads with i >= nb contribute zeros but still take part in the shuffles.
template <int CW>
__device__ inline void tile_prod(const zd *__restrict__ T, const zd *v, int nb,
                                 const SolveGeom &sg, int i, int g, int shape, zd *acc) {
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = zmake(0, 0);
    if (i < nb) {
        int k0 = g * sg.klen;
        int k1 = min(nb, k0 + sg.klen);
        if (shape == kLower) k1 = min(k1, i + 1);
        else if (shape == kUpper) k0 = max(k0, i);
        const zd *tp = T + i;
        for (int kb = k0; kb < k1; kb += kSeg) {
            zd t[kSeg];
#pragma unroll
            for (int u = 0; u < kSeg; ++u)
                t[u] = (kb + u < k1) ? tp[int64_t(kb + u) * nb] : zmake(0, 0);
#pragma unroll
            for (int u = 0; u < kSeg; ++u) {
                if (kb + u < k1) {
                    const zd *vr = v + (kb + u) * CW;
#pragma unroll
                    for (int c = 0; c < CW; ++c) zfma(acc[c], t[u], vr[c]);
                }
            }
        }
    }
    for (int off = sg.G / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            acc[c].x += __shfl_xor(acc[c].x, off, 64);
            acc[c].y += __shfl_xor(acc[c].y, off, 64);
        }
    }
}

template <int CW, int NT>
__global__ __launch_bounds__(NT) void band_solve_kernel(SolveArgs a) {
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
    const SolveGeom sg = solve_geom(nb, NT);
    const int wave = tid / 64, lane = tid % 64;
    const int i = wave * sg.rows_per_wave + lane / sg.G;    // output row of this thread
    const int g = lane % sg.G;
    const bool writer = (g == 0) && (i < nb);

    extern __shared__ unsigned char smem_raw[];
    zd *win = reinterpret_cast<zd *>(smem_raw);   // [2nb][CW]
    zd *win2 = win + 2 * nb * CW;                 // [2nb][CW]
    zd *ybuf = win2 + 2 * nb * CW;                // [nb][CW]
    zd *ring = ybuf + nb * CW;                    // [3][nb][CW]

    zd *yp = a.ypart + int64_t(pole) * a.npad * a.ncols;
    zd *xp = a.xpart + int64_t(pole) * a.npad * a.ncols;
    const zd *tiles = a.tiles + int64_t(pole) * nblk * 5 * te;
    const int32_t *perm = a.perm + int64_t(pole) * nblk * 2 * nb;

    // L2 prefetch: the workgroups of this pole that share an XCD (workgroups are
    // dealt to the 8 XCDs round-robin) split the next step's tiles between them and
    // touch one element per 128-byte line, so the tile reads of the next step hit L2.
    const int nslices = (a.ncols + CW - 1) / CW;
    const int spread = (8 % p == 0) ? 8 / p : 1;          // XCDs one pole is spread over
    const int prank = slice / spread;
    const int pcount = (nslices + spread - 1) / spread;
    double sink = 0.0;
    auto touch = [&](const zd *base, int64_t elems) {
        const int64_t lines = (elems + 7) / 8;              // 8 complex per 128-byte line
        const int64_t per = (lines + pcount - 1) / pcount;
        const int64_t l0 = int64_t(prank) * per, l1 = min(lines, l0 + per);
        for (int64_t ln = l0 + tid; ln < l1; ln += NT) sink += base[ln * 8].x;
    };

    // right-hand-side rows of block blk for element e of the [nb][CW] block
    auto rhs_elem = [&](int blk, int e) {
        int r = e / CW, c = e % CW;
        int64_t row = int64_t(blk) * nb + r;
        zd v = zmake(0, 0);
        if (row < a.n && c < ncw) {
            v = a.X[row + int64_t(c0 + c) * a.ldx];
            if (a.bdiag) v = zmul(a.bdiag[row], v);
        }
        return v;
    };
    constexpr int RPT = (256 * CW + NT - 1) / NT;        // rhs elements per thread (nb <= 256)
    zd pre[RPT];
    auto prefetch_rhs = [&](int blk) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int e = tid + q * NT;
            pre[q] = (blk < nblk && e < nb * CW) ? rhs_elem(blk, e) : zmake(0, 0);
        }
    };
    auto store_rhs = [&](zd *dst) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int e = tid + q * NT;
            if (e < nb * CW) dst[e] = pre[q];
        }
    };

    zd acc[CW];
    // ---------------- forward sweep
    prefetch_rhs(0);
    store_rhs(win);
    prefetch_rhs(1);
    for (int k = 0; k < nblk; ++k) {
        const bool last = (k + 1 == nblk);
        if (!last) store_rhs(win + nb * CW);                 // b_{k+1}
        prefetch_rhs(k + 2);                                 // b_{k+2}, used next step
        if (!last) touch(tiles + int64_t(k + 1) * 5 * te, 2 * te);   // Linv, L21 of step k+1
        __syncthreads();
        const int rows = last ? nb : 2 * nb;
        const int32_t *pk = perm + int64_t(k) * 2 * nb;
        for (int e = tid; e < rows * CW; e += NT) {
            int r = e / CW, c = e % CW;
            win2[e] = win[pk[r] * CW + c];
        }
        __syncthreads();
        const zd *Tk = tiles + int64_t(k) * 5 * te;
        tile_prod<CW>(Tk, win2, nb, sg, i, g, kLower, acc);      // y_k = Linv w_top
        if (writer) {
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                ybuf[i * CW + c] = acc[c];
                if (c < ncw) yp[int64_t(k) * nb + i + int64_t(c0 + c) * a.npad] = acc[c];
            }
        }
        __syncthreads();
        if (!last) {
            tile_prod<CW>(Tk + te, ybuf, nb, sg, i, g, kFull, acc);   // t_{k+1} = w_bot - L21 y_k
            if (writer) {
#pragma unroll
                for (int c = 0; c < CW; ++c) win[i * CW + c] = zsub(win2[(nb + i) * CW + c], acc[c]);
            }
        }
        __syncthreads();
    }
    // ---------------- backward sweep
    for (int e = tid; e < 3 * nb * CW; e += NT) ring[e] = zmake(0, 0);
    touch(tiles + int64_t(nblk - 1) * 5 * te + 2 * te, 3 * te);
    zd ynext[CW];
    auto load_y = [&](int k, zd *dst) {
#pragma unroll
        for (int c = 0; c < CW; ++c)
            dst[c] = (writer && k >= 0 && c < ncw) ? yp[int64_t(k) * nb + i + int64_t(c0 + c) * a.npad]
                                                  : zmake(0, 0);
    };
    load_y(nblk - 1, ynext);
    __syncthreads();
    for (int k = nblk - 1; k >= 0; --k) {
        zd *xk = ring + (k % 3) * nb * CW;
        const zd *xk1 = ring + ((k + 1) % 3) * nb * CW;
        const zd *xk2 = ring + ((k + 2) % 3) * nb * CW;
        const zd *Tk = tiles + int64_t(k) * 5 * te;
        zd y[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) y[c] = ynext[c];
        load_y(k - 1, ynext);                                       // y_{k-1}, used next step
        if (k > 0) touch(tiles + int64_t(k - 1) * 5 * te + 2 * te, 3 * te);   // Uinv, U1, U2 of k-1
        // v = y_k - U1 x_{k+1} - U2 x_{k+2}
        zd acc2[CW];
        tile_prod<CW>(Tk + 3 * te, xk1, nb, sg, i, g, kFull, acc);
        tile_prod<CW>(Tk + 4 * te, xk2, nb, sg, i, g, kLower, acc2);
        if (writer) {
#pragma unroll
            for (int c = 0; c < CW; ++c) ybuf[i * CW + c] = zsub(zsub(y[c], acc[c]), acc2[c]);
        }
        __syncthreads();
        tile_prod<CW>(Tk + 2 * te, ybuf, nb, sg, i, g, kUpper, acc);     // x_k = Uinv v
        if (writer) {
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                xk[i * CW + c] = acc[c];
                if (c < ncw) xp[int64_t(k) * nb + i + int64_t(c0 + c) * a.npad] = zmul(wgt, acc[c]);
            }
        }
        __syncthreads();
    }
    // keep the prefetch loads alive without storing anything real (n is never negative)
    if (a.n < 0) ybuf[0] = zmake(sink, 0.0);
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
    auto panel_lds = [&](int nc) {
        return size_t(2 * nb * nc + nc * nb) * sizeof(zd) + (nb + 4 * nc) * sizeof(int) +
               (kThreads / 64) * (sizeof(double) + sizeof(int));
    };
    const int nc = panel_lds(16) <= size_t(P.max_lds) ? 16 : (panel_lds(8) <= size_t(P.max_lds) ? 8 : 4);
    // update kernel LDS: permuted columns [2nb][cpw] + one L column block [2nb][16]
    const int cpw = (size_t(2 * nb) * (16 + 16) * sizeof(zd) <= size_t(P.max_lds)) ? 16 : 8;
    const size_t upd_lds = size_t(2 * nb) * (cpw + 16) * sizeof(zd);
    hipLaunchKernelGGL(band_window_init_kernel, dim3(p), dim3(256), 0, s, a);
    int buf = 0;
    for (int k = 0; k < a.nblk; ++k) {
        if (nc == 16)
            hipLaunchKernelGGL(band_panel_kernel<16>, dim3(p), dim3(kThreads), panel_lds(16), s, a, k, buf);
        else if (nc == 8)
            hipLaunchKernelGGL(band_panel_kernel<8>, dim3(p), dim3(kThreads), panel_lds(8), s, a, k, buf);
        else
            hipLaunchKernelGGL(band_panel_kernel<4>, dim3(p), dim3(kThreads), panel_lds(4), s, a, k, buf);
        if (cpw == 16)
            hipLaunchKernelGGL(band_update_kernel<16>, dim3(2 * nb / 16, p), dim3(kThreads), upd_lds, s, a, k, buf);
        else
            hipLaunchKernelGGL(band_update_kernel<8>, dim3(2 * nb / 8, p), dim3(kThreads), upd_lds, s, a, k, buf);
        buf ^= 1;
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
    // win + win2 (2nb each) + ybuf (nb) + ring (3nb), all x cw
    return size_t(2 * nb * cw * 2 + nb * cw + 3 * nb * cw) * sizeof(zd);
}

template <int CW>
static hipError_t launch_solve_cw(const SolveArgs &a, hipStream_t s) {
    const int slices = (a.ncols + CW - 1) / CW;
    // more columns per workgroup -> more accumulator registers -> fewer threads
    constexpr int NT = CW <= 2 ? 1024 : 512;
    hipLaunchKernelGGL((band_solve_kernel<CW, NT>), dim3(slices * a.p), dim3(NT),
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
    hipEvent_t ev0 = nullptr;
    P.prof.record_begin(s, ev0);
    switch (cw) {
        case 1: e = launch_solve_cw<1>(a, s); break;
        case 2: e = launch_solve_cw<2>(a, s); break;
        case 4: e = launch_solve_cw<4>(a, s); break;
        default: e = launch_solve_cw<8>(a, s); break;
    }
    if (e != hipSuccess) return e;
    P.prof.record_end(s, ev0, ncols, 0);
    int64_t tot = P.n * ncols;
    hipLaunchKernelGGL(pole_sum_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, P.xpart, a.p,
                       a.npad, P.n, ncols, Z, ldz);
    return hipGetLastError();
}
