// Dense and sparse block kernels of the composite-rule filter (gfx950):
//   * tall-skinny complex products V^H W (split over rows, fixed-order reduction)
//     and W - V H on the FP64 matrix cores, used by block Gram-Schmidt in the block-Arnoldi process
//     (Sec. 3.2, multi-shift GMRES) and by the projections of HSRR (Sec. 2.1);
//   * Cholesky of small Gram matrices (CholeskyQR orthonormalisation, the
//     "orth" of Alg. SIsketch);
//   * the per-shift least-squares updates of multi-shift block GMRES: for every
//     shift s_j the block Hessenberg matrix H - s_j I~ is reduced to triangular
//     form one block column per step with Householder reflectors, giving the
//     residual of every column and shift after each step;
//   * CSR times block, column norms, start-block generation.
//
// Batched kernels take an optional index map: operand X of batch entry t lives at
// base_X + (mapped_X ? map[t] : t) * stride_X.  The Krylov sub-blocks that are
// still active are addressed this way without compacting their storage.
#include "rf_common.h"

namespace {

constexpr int TM = 64, TN = 64, TK = 16, GT = 256;

__device__ inline int64_t bidx(const int *map, int flags, int bit, int t) {
    return (map && (flags & bit)) ? map[t] : t;
}

// Sums over aligned groups of 8 (or 4) lanes with DPP lane moves (no LDS round trip);
// every lane of a group ends with the same value.
__device__ __attribute__((always_inline)) inline double dpp_move(double v, int ctrl_sel) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int olo, ohi;
    switch (ctrl_sel) {
        case 0:  // quad_perm [1,0,3,2]: lane xor 1
            olo = __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false);
            ohi = __builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false);
            break;
        case 1:  // quad_perm [2,3,0,1]: lane xor 2
            olo = __builtin_amdgcn_update_dpp(lo, lo, 0x4E, 0xF, 0xF, false);
            ohi = __builtin_amdgcn_update_dpp(hi, hi, 0x4E, 0xF, 0xF, false);
            break;
        default:  // row_half_mirror: lane 7 - i within each group of 8
            olo = __builtin_amdgcn_update_dpp(lo, lo, 0x141, 0xF, 0xF, false);
            ohi = __builtin_amdgcn_update_dpp(hi, hi, 0x141, 0xF, 0xF, false);
            break;
    }
    return __hiloint2double(ohi, olo);
}
__device__ __attribute__((always_inline)) inline double group4_sum(double v) {
    v += dpp_move(v, 0);
    v += dpp_move(v, 1);
    return v;
}
__device__ __attribute__((always_inline)) inline double group8_sum(double v) {
    v = group4_sum(v);
    v += dpp_move(v, 2);      // the other quad of the group holds the other half
    return v;
}


// ---------------------------------------------------------------------------
// Tall-skinny products on the FP64 matrix cores.
//   C_part[chunk] = A[rows of chunk]^H B[rows of chunk]     (split over rows, then a
//   fixed-order reduction; grid (ceil(m / 16 TMB), ceil(k / 16 TNB), batch * nchunks))
//   C = alpha A B + beta C                                    (64-row tiles)
// v_mfma_f64_16x16x4f64 takes a 16 x 4 block of A with element (i, k) in lane i + 16 k,
// a 4 x 16 block of B with element (k, j) in lane j + 16 k, and accumulates the 16 x 16
// product with element (4 r + l / 16, l % 16) in slot r of lane l.  A complex block
// product is four real ones, real and imaginary parts accumulated separately; each
// wave owns 16 x 16 output blocks.  Slabs of TKS rows (columns) go through LDS, the
// next slab read into registers while the current one is multiplied, so global
// latency is paid once per chunk.  Output tiles are 32 wide when an operand is one
// Krylov sub-block (b = 32), so no multiply-add is spent on padding.
// ---------------------------------------------------------------------------
constexpr int TKS = 32;
typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __attribute__((always_inline)) inline dv4 mfma_f64(double a, double b, dv4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int TMB, int TNB>
__global__ __launch_bounds__(GT) void gemm_cn_mfma_kernel(
    int64_t n, int m, int k, const zd *__restrict__ A, int64_t lda, int64_t sA,
    const zd *__restrict__ B, int64_t ldb, int64_t sB, zd *__restrict__ part, int nchunks,
    int64_t chunk, const int *map, int flags) {
    constexpr int TMT = 16 * TMB, TNT = 16 * TNB;
    constexpr int BPW = TMB * TNB / 4;                          // output blocks per wave
    constexpr int LA = TKS * TMT / GT, LB = TKS * TNT / GT;
    static_assert(TMB * TNB % 4 == 0, "four waves share the output blocks");
    const int bt = blockIdx.z / nchunks, ch = blockIdx.z % nchunks;
    const int m0 = blockIdx.x * TMT, k0 = blockIdx.y * TNT;
    A += bidx(map, flags, kMapA, bt) * sA;
    B += bidx(map, flags, kMapB, bt) * sB;
    const int64_t r0 = int64_t(ch) * chunk;
    const int64_t r1 = min(n, r0 + chunk);
    __shared__ zd As[TKS][TMT + 1];
    __shared__ zd Bs[TKS][TNT + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    zd ra[LA], rb[LB];
    // rows are the fastest index of a slab element: coalesced column runs
    auto fetch = [&](int64_t rr) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int e = tid + q * GT, i = e % TKS, c = e / TKS;
            const int64_t row = rr + i;
            ra[q] = (row < r1 && m0 + c < m) ? A[row + int64_t(m0 + c) * lda] : zmake(0, 0);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + q * GT, i = e % TKS, c = e / TKS;
            const int64_t row = rr + i;
            rb[q] = (row < r1 && k0 + c < k) ? B[row + int64_t(k0 + c) * ldb] : zmake(0, 0);
        }
    };
    dv4 accR[BPW], accI[BPW];
#pragma unroll
    for (int t = 0; t < BPW; ++t) { accR[t] = dv4{0, 0, 0, 0}; accI[t] = dv4{0, 0, 0, 0}; }
    if (r0 < r1) fetch(r0);
    for (int64_t rr = r0; rr < r1; rr += TKS) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int e = tid + q * GT;
            As[e % TKS][e / TKS] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + q * GT;
            Bs[e % TKS][e / TKS] = rb[q];
        }
        __syncthreads();
        if (rr + TKS < r1) fetch(rr + TKS);
#pragma unroll
        for (int ks = 0; ks < TKS / 4; ++ks) {
            const int row = ks * 4 + lk;
#pragma unroll
            for (int t = 0; t < BPW; ++t) {
                const int blk = wave * BPW + t, bi = blk / TNB, bj = blk % TNB;
                const zd a = As[row][bi * 16 + li];       // conj(A)^T: (i, k) = conj(A[k][i])
                const zd b = Bs[row][bj * 16 + li];
                accR[t] = mfma_f64(a.x, b.x, accR[t]);
                accR[t] = mfma_f64(a.y, b.y, accR[t]);
                accI[t] = mfma_f64(a.x, b.y, accI[t]);
                accI[t] = mfma_f64(-a.y, b.x, accI[t]);
            }
        }
        __syncthreads();
    }
    zd *P = part + (int64_t(bt) * nchunks + ch) * int64_t(m) * k;
#pragma unroll
    for (int t = 0; t < BPW; ++t) {
        const int blk = wave * BPW + t, bi = blk / TNB, bj = blk % TNB;
        const int kj = k0 + bj * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mi = m0 + bi * 16 + 4 * r + lk;
            if (mi < m && kj < k) P[mi + int64_t(kj) * m] = zmake(accR[t][r], accI[t][r]);
        }
    }
}

// C = alpha * sum_chunks part + beta * C   (fixed summation order).  Four lanes per
// output: lane q sums chunks [q P, (q+1) P) in order with all of its reads in flight
// at once, then the four sums are added in a fixed tree by DPP (the partials were
// written from every XCD, so each read is a far round trip).
__global__ void gemm_cn_reduce_kernel(int m, int k, const zd *part, int nchunks, zd alpha,
                                      zd beta, zd *C, int64_t ldc, int64_t sC, int batch,
                                      const int *map, int flags) {
    const int64_t gt = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t e = gt >> 2;
    const int q = int(gt & 3);
    const int64_t mk = int64_t(m) * k;
    const bool ok = e < mk * batch;          // the same for the four lanes of an output
    const int64_t ee = ok ? e : 0;
    const int bt = int(ee / mk);
    const int64_t r = ee % mk;
    const int mi = int(r % m), kj = int(r / m);
    const zd *P = part + int64_t(bt) * nchunks * mk + r;
    const int per = (nchunks + 3) / 4;
    const int c0 = q * per, c1 = min(nchunks, c0 + per);
    zd s = zmake(0, 0);
    for (int c = c0; c < c1; c += 16) {
        zd t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = (c + u < c1) ? P[int64_t(c + u) * mk] : zmake(0, 0);
#pragma unroll
        for (int u = 0; u < 16; ++u) s = zadd(s, t[u]);
    }
    s.x = group4_sum(s.x);
    s.y = group4_sum(s.y);
    if (ok && q == 0) {
        zd *cp = C + bidx(map, flags, kMapC, bt) * sC + mi + int64_t(kj) * ldc;
        zd out = zmul(alpha, s);
        if (beta.x != 0.0 || beta.y != 0.0) zfma(out, beta, *cp);
        *cp = out;
    }
}

// C (n x k) = alpha A (n x m) B (m x k) + beta C, grid (ceil(n / 64), ceil(k / 16 TNB),
// batch): wave w owns rows 16 w .. 16 w + 15 of the 64-row tile and all TNB column blocks.
template <int TNB>
__global__ __launch_bounds__(GT) void gemm_nn_mfma_kernel(int64_t n, int m, int k, zd alpha,
                                                          const zd *__restrict__ A, int64_t lda,
                                                          int64_t sA, const zd *__restrict__ B,
                                                          int64_t ldb, int64_t sB, zd beta, zd *C,
                                                          int64_t ldc, int64_t sC, const int *map,
                                                          int flags) {
    constexpr int TNT = 16 * TNB;
    constexpr int LA = TKS * TM / GT, LB = TKS * TNT / GT;
    const int bt = blockIdx.z;
    const int64_t n0 = int64_t(blockIdx.x) * TM;
    const int k0 = blockIdx.y * TNT;
    A += bidx(map, flags, kMapA, bt) * sA;
    B += bidx(map, flags, kMapB, bt) * sB;
    C += bidx(map, flags, kMapC, bt) * sC;
    __shared__ zd As[TKS][TM + 1];
    __shared__ zd Bs[TKS][TNT + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    zd ra[LA], rb[LB];
    auto fetch = [&](int kk) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int e = tid + q * GT, r = e % TM, i = e / TM;   // rows of A fastest
            const int64_t row = n0 + r;
            ra[q] = (row < n && kk + i < m) ? A[row + int64_t(kk + i) * lda] : zmake(0, 0);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + q * GT, i = e % TKS, c = e / TKS;  // rows of B fastest
            rb[q] = (kk + i < m && k0 + c < k) ? B[(kk + i) + int64_t(k0 + c) * ldb] : zmake(0, 0);
        }
    };
    dv4 accR[TNB], accI[TNB];
#pragma unroll
    for (int t = 0; t < TNB; ++t) { accR[t] = dv4{0, 0, 0, 0}; accI[t] = dv4{0, 0, 0, 0}; }
    if (m > 0) fetch(0);
    for (int kk = 0; kk < m; kk += TKS) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int e = tid + q * GT;
            As[e / TM][e % TM] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + q * GT;
            Bs[e % TKS][e / TKS] = rb[q];
        }
        __syncthreads();
        if (kk + TKS < m) fetch(kk + TKS);
#pragma unroll
        for (int ks = 0; ks < TKS / 4; ++ks) {
            const int i = ks * 4 + lk;
            const zd a = As[i][wave * 16 + li];               // A block (row li, column lk)
#pragma unroll
            for (int t = 0; t < TNB; ++t) {
                const zd b = Bs[i][t * 16 + li];               // B block (row lk, column li)
                accR[t] = mfma_f64(a.x, b.x, accR[t]);
                accR[t] = mfma_f64(-a.y, b.y, accR[t]);
                accI[t] = mfma_f64(a.x, b.y, accI[t]);
                accI[t] = mfma_f64(a.y, b.x, accI[t]);
            }
        }
        __syncthreads();
    }
    const bool use_beta = (beta.x != 0.0 || beta.y != 0.0);
#pragma unroll
    for (int t = 0; t < TNB; ++t) {
        const int col = k0 + t * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = n0 + wave * 16 + 4 * r + lk;
            if (row < n && col < k) {
                zd *cp = C + row + int64_t(col) * ldc;
                zd out = zmul(alpha, zmake(accR[t][r], accI[t][r]));
                if (use_beta) zfma(out, beta, *cp);
                *cp = out;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Cholesky S = R^H R (R upper) of a batch of k x k Hermitian matrices (leading
// dimension k), then Rinv = R^{-1}.  The diagonal is raised by shift_rel * max_i S_ii
// before factoring (shifted CholeskyQR).  status[t] = 1 + the first column whose
// pivot is not positive; dratio[t] = min_i R_ii / max_i R_ii (condition estimate).
// ---------------------------------------------------------------------------
// Register version for k <= K (K = 32 or 64): thread (i = tid % K, g = tid / K) holds
// row i, columns g CPT .. g CPT + CPT - 1 of the matrix being reduced and of X.
//   Cholesky, right-looking: before step j every thread reads column j (published in
//   LDS by its owners at the end of step j - 1), scales its element of column j by
//   1 / sqrt(d_j) and takes the rank-one update of its elements right of column j;
//   the owners of column j + 1 then publish it.
//   X = L^{-1} in the same steps (right-looking forward substitution on the identity):
//   row j of X is final once the steps before j have been taken, so its owners
//   publish it beside column j; step j scales it by 1 / L_jj and every row below
//   subtracts L_ij times it.  Per element these are the operations, in the order, of a
//   separate substitution pass after the factorization, which would take K more
//   steps.  Column and row buffers alternate by step parity: one barrier per step.
// Rows and columns past k are the identity and take no part.
template <int K, int NT>
__global__ __launch_bounds__(NT) void chol_inv_reg_kernel(int k, const zd *S, int64_t sS,
                                                          zd *Rout, int64_t sR, zd *Rinv,
                                                          int64_t sRi, int *status,
                                                          double *dratio, double shift_rel,
                                                          const int *map, int flags) {
    constexpr int NCG = NT / K, CPT = K / NCG;
    const int bt = blockIdx.x;
    const zd *Sg = S + bidx(map, flags, kMapA, bt) * sS;
    zd *Rg = Rout + bidx(map, flags, kMapB, bt) * sR;
    zd *Rig = Rinv + bidx(map, flags, kMapC, bt) * sRi;
    const int tid = threadIdx.x, i = tid % K, g = tid / K, c0 = g * CPT;
    __shared__ zd colb[2][K];                // column j of the matrix being reduced
    __shared__ zd rowb[2][K];                // row j of X
    __shared__ double sdiag[K];              // L_jj
    __shared__ double s_shift;
    __shared__ int s_bad;
    zd a[CPT], x[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int l = c0 + q;
        a[q] = (i < k && l < k) ? Sg[i + int64_t(l) * k] : zmake(i == l ? 1.0 : 0.0, 0.0);
        x[q] = zmake(l == i ? 1.0 : 0.0, 0.0);
    }
    // the diagonal for the shift (one element per thread, read in parallel)
    if (tid < K) sdiag[tid] = (tid < k) ? Sg[tid + int64_t(tid) * k].x : 0.0;
    // column 0 and row 0 of X published by their owners
    if (g == 0) colb[0][i] = a[0];
    if (i == 0) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) rowb[0][c0 + q] = x[q];
    }
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        for (int r = 0; r < k; ++r) mx = fmax(mx, sdiag[r]);
        s_shift = shift_rel * mx;
        s_bad = 0;
    }
    __syncthreads();
    const double shift = s_shift;
    // column j = jb CPT + jj: the group index jb is a loop variable and jj a constant
    // of the unrolled inner loop, so every register index below is a constant
#pragma unroll 1
    for (int jb = 0; jb < NCG; ++jb) {
#pragma unroll
        for (int jj = 0; jj < CPT; ++jj) {
            const int j = jb * CPT + jj, par = jj & 1;     // CPT is even: parity of j
            const zd *cj = colb[par];
            const zd *xj = rowb[par];
            double d = cj[j].x + (j < k ? shift : 0.0);
            if (!(d > 0.0)) {
                if (tid == 0 && s_bad == 0) s_bad = j + 1;
                d = 1.0;
            }
            const double sq = sqrt(d), rs = 1.0 / sq, rd = 1.0 / d;
            if (tid == 0) sdiag[j] = sq;
            const zd ci = cj[i];
            zd cl[CPT], xr[CPT];                       // all reads issued before any use
#pragma unroll
            for (int q = 0; q < CPT; ++q) { cl[q] = cj[c0 + q]; xr[q] = xj[c0 + q]; }
            const zd cir = zmake(ci.x * rd, ci.y * rd);
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int l = c0 + q;
                // A_il -= A_ij conj(A_lj) / d right of column j (lower triangle only)
                const bool right = (g > jb) || (g == jb && q > jj);
                if (right && l <= i) {
                    a[q].x -= cir.x * cl[q].x + cir.y * cl[q].y;
                    a[q].y -= cir.y * cl[q].x - cir.x * cl[q].y;
                }
            }
            const zd lij = (i > j) ? zmake(ci.x * rs, ci.y * rs) : zmake(0, 0);
            if (g == jb) a[jj] = (i == j) ? zmake(sq, 0.0) : lij;
            // X: row j scaled by 1 / L_jj; the rows below subtract L_ij times it (the
            // rows at or above j take it times zero)
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const zd xs = zmake(xr[q].x * rs, xr[q].y * rs);
                if (i == j) x[q] = xs;
                else zfms(x[q], lij, xs);
            }
            // publish column j + 1 and row j + 1 of X
            if (jj + 1 < CPT) {
                if (g == jb) colb[par ^ 1][i] = a[jj + 1 < CPT ? jj + 1 : 0];
            } else if (g == jb + 1) {
                colb[par ^ 1][i] = a[0];
            }
            if (i == j + 1) {
#pragma unroll
                for (int q = 0; q < CPT; ++q) rowb[par ^ 1][c0 + q] = x[q];
            }
            __syncthreads();
        }
    }
    // R = L^H (upper), Rinv = X^H
    if (i < k) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int l = c0 + q;
            if (l < k) {
                Rg[l + int64_t(i) * k] = (l <= i) ? zconj(a[q]) : zmake(0, 0);
                Rig[l + int64_t(i) * k] = (l <= i) ? zconj(x[q]) : zmake(0, 0);
            }
        }
    }
    if (tid == 0) {
        double mn = 1e300, mx = 0.0;
        for (int r = 0; r < k; ++r) { mn = fmin(mn, sdiag[r]); mx = fmax(mx, sdiag[r]); }
        if (status) status[bt] = s_bad;
        if (dratio) dratio[bt] = (mx > 0.0) ? mn / mx : 0.0;
    }
}

// Global-memory version for k > 64 (one workgroup per matrix, S overwritten).
__global__ __launch_bounds__(GT) void chol_inv_kernel(int k, zd *S, int64_t sS, zd *Rout,
                                                      int64_t sR, zd *Rinv, int64_t sRi,
                                                      int *status, double *dratio,
                                                      double shift_rel) {
    const int bt = blockIdx.x;
    zd *A = S + bt * sS;
    zd *R = Rout + bt * sR;
    zd *Ri = Rinv + bt * sRi;
    const int tid = threadIdx.x;
    __shared__ int bad;
    __shared__ double shift;
    __shared__ double djj;
    if (tid == 0) {
        bad = 0;
        double mx = 0.0;
        for (int i = 0; i < k; ++i) mx = fmax(mx, A[i + int64_t(i) * k].x);
        shift = shift_rel * mx;
    }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (tid == 0) {
            double d = A[j + int64_t(j) * k].x + shift;
            if (!(d > 0.0)) { if (!bad) bad = j + 1; d = 1.0; }
            djj = sqrt(d);
            A[j + int64_t(j) * k] = zmake(djj, 0.0);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < k; i += GT) A[i + int64_t(j) * k] = zscale(A[i + int64_t(j) * k], 1.0 / djj);
        __syncthreads();
        const int rem = k - j - 1;
        for (int e = tid; e < rem * rem; e += GT) {
            int i = j + 1 + e % rem, l = j + 1 + e / rem;
            if (l > i) continue;
            zd v = A[i + int64_t(l) * k];
            zd lij = A[i + int64_t(j) * k], llj = A[l + int64_t(j) * k];
            v.x -= lij.x * llj.x + lij.y * llj.y;
            v.y -= lij.y * llj.x - lij.x * llj.y;
            if (i == l) v.y = 0.0;
            A[i + int64_t(l) * k] = v;
        }
        __syncthreads();
    }
    for (int e = tid; e < k * k; e += GT) {
        int i = e % k, j = e / k;
        R[i + int64_t(j) * k] = (i <= j) ? zconj(A[j + int64_t(i) * k]) : zmake(0, 0);
        Ri[i + int64_t(j) * k] = zmake(0, 0);
    }
    __syncthreads();
    // Rinv: row by row from the bottom, all columns in parallel
    for (int r = k - 1; r >= 0; --r) {
        for (int c = r + tid; c < k; c += GT) {
            zd v = (r == c) ? zmake(1.0, 0.0) : zmake(0, 0);
            for (int q = r + 1; q <= c; ++q) zfms(v, R[r + int64_t(q) * k], Ri[q + int64_t(c) * k]);
            Ri[r + int64_t(c) * k] = zscale(v, 1.0 / R[r + int64_t(r) * k].x);
        }
        __syncthreads();
    }
    if (tid == 0) {
        double mn = 1e300, mx = 0.0;
        for (int i = 0; i < k; ++i) { double d = R[i + int64_t(i) * k].x; mn = fmin(mn, d); mx = fmax(mx, d); }
        if (status) status[bt] = bad;
        if (dratio) dratio[bt] = (mx > 0.0) ? mn / mx : 0.0;
    }
}

// C[map] (m x k block, ldc) += alpha * Aop (m x k, lda), batched
__global__ void add_block_kernel(int m, int k, zd alpha, const zd *A, int64_t lda, int64_t sA,
                                 zd *C, int64_t ldc, int64_t sC, int batch, const int *map,
                                 int flags) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t mk = int64_t(m) * k;
    if (e >= mk * batch) return;
    int bt = int(e / mk);
    int64_t r = e % mk;
    int i = int(r % m), j = int(r / m);
    const zd *ap = A + bidx(map, flags, kMapA, bt) * sA + i + int64_t(j) * lda;
    zd *cp = C + bidx(map, flags, kMapC, bt) * sC + i + int64_t(j) * ldc;
    zd v = *cp;
    zfma(v, alpha, *ap);
    *cp = v;
}

// dst[map] (n x ncols) = src[map]   (batched column-block copy)
__global__ void copy_block_kernel(int64_t n, int ncols, const zd *src, int64_t lds, int64_t sS,
                                  zd *dst, int64_t ldd, int64_t sD, int batch, const int *map,
                                  int flags) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t per = n * ncols;
    if (e >= per * batch) return;
    int bt = int(e / per);
    int64_t r = e % per;
    int64_t i = r % n, c = r / n;
    dst[bidx(map, flags, kMapC, bt) * sD + i + c * ldd] = src[bidx(map, flags, kMapA, bt) * sS + i + c * lds];
}

__global__ void copy_cols_kernel(int64_t n, int ncols, const zd *src, int64_t lds, zd *dst,
                                 int64_t ldd) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    dst[r + c * ldd] = src[r + c * lds];
}

// Y = M X for CSR M (one thread per (row, column))
__global__ void spmm_kernel(int64_t n, int ncols, const int32_t *rp, const int32_t *ci,
                            const zd *val, const zd *X, int64_t ldx, zd *Y, int64_t ldy) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    zd acc = zmake(0, 0);
    for (int q = rp[r]; q < rp[r + 1]; ++q) zfma(acc, val[q], X[ci[q] + c * ldx]);
    Y[r + c * ldy] = acc;
}

__global__ void axpby_kernel(int64_t n, int ncols, zd alpha, const zd *X, int64_t ldx, zd beta,
                             const zd *Y, int64_t ldy, zd *Z, int64_t ldz) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    zd v = zmul(alpha, X[r + c * ldx]);
    zfma(v, beta, Y[r + c * ldy]);
    Z[r + c * ldz] = v;
}

// out[c] = || X[:, c] - lam[c] * Y[:, c] ||_2     (one workgroup per column)
__global__ __launch_bounds__(GT) void colnorm_kernel(int64_t n, const zd *X, int64_t ldx,
                                                     const zd *Y, int64_t ldy, const zd *lam,
                                                     double *out) {
    const int c = blockIdx.x;
    const zd *x = X + c * ldx;
    const zd *y = Y ? Y + c * ldy : nullptr;
    const zd l = lam ? lam[c] : zmake(0, 0);
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += GT) {
        zd v = x[r];
        if (y) zfms(v, l, y[r]);
        s += zabs2(v);
    }
    __shared__ double red[GT];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = GT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sqrt(red[0]);
}

__global__ void scale_cols_kernel(int64_t n, int ncols, zd *X, int64_t ldx, const double *inv) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    X[r + c * ldx] = zscale(X[r + c * ldx], inv[c]);
}

// dst[c] = 1 / src[c] for positive entries, else `other` (column scalings computed
// on the device, so that no host round trip sits between the norms and their use)
__global__ void inv_pos_kernel(int m, const double *src, double *dst, double other) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < m) dst[c] = src[c] > 0.0 ? 1.0 / src[c] : other;
}

// splitmix64-based counter generator: element (r, c) draws from counter r + c*n
__device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__global__ void gaussian_kernel(int64_t n, int ncols, zd *X, int64_t ldx, uint64_t seed) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    uint64_t h1 = splitmix64(seed * 0x632BE59BD9B4E019ull + 2 * uint64_t(e));
    uint64_t h2 = splitmix64(seed * 0x632BE59BD9B4E019ull + 2 * uint64_t(e) + 1);
    double u1 = (double((h1 >> 11) + 1)) * (1.0 / 9007199254740993.0);
    double u2 = double(h2 >> 11) * (1.0 / 9007199254740992.0);
    double rad = sqrt(-2.0 * log(u1)) * 0.7071067811865476;
    double ang = 6.283185307179586 * u2;
    X[r + c * ldx] = zmake(rad * cos(ang), rad * sin(ang));
}

// ---------------------------------------------------------------------------
// Multi-shift block GMRES least squares.
// For shift s_l and sub-block sb, at block-Arnoldi step j the new block column
// of H - s_l I~ (rows 0..(j+2)b) is rotated by the stored unitary blocks Q_0..Q_{j-1}
// (each acting on two block rows), then a Householder QR of its bottom 2b x b block
// gives R_jj and Q_j (stored explicitly, 2b x 2b).  The right-hand side E1 R0 is
// rotated by Q_j^H; the norms of its last b rows are the residuals.
// One workgroup per (shift, active sub-block).  The column is streamed through a
// 2b x b window in LDS: rows come straight from H (the shift subtracted on the fly),
// each rotation's finished top block row goes straight into R, and Q_{i+1} is
// loaded into registers while Q_i is applied.
// ---------------------------------------------------------------------------
struct LsArgs {
    int b, mmax, j, nq;
    const zd *shifts;
    const zd *H; int64_t ldh, sH;       // block Hessenberg per sub-block
    zd *Q; zd *R; zd *G; zd *work;
    double *resid;                      // [nq][nsub][b]
    const double *r0norm;               // [nsub][b] column norms of the start block
    const int *active;
    int nsub;
};

__device__ inline int64_t ls_off(int l, int sb, int nsub, int64_t per) {
    return (int64_t(l) * nsub + sb) * per;
}

// out (2b x b, LDS, ld 2b) = Q^H in, with Q in LDS (ld ldq, conjugated on use) and
// in (2b x b, LDS, ld 2b).  Each thread computes a 2 x 4 block of out (rows r, r + b;
// columns 4q..4q+3), so every LDS read feeds several multiply-adds (b < 4: one
// element per thread).
__device__ inline void apply_qh(const zd *Qs, int ldq, const zd *in, zd *out, int b) {
    const int m2 = 2 * b;
    if (b % 4 != 0) {
        for (int e = threadIdx.x; e < m2 * b; e += GT) {
            const int r = e % m2, c = e / m2;
            zd acc = zmake(0, 0);
            for (int t = 0; t < m2; ++t) zfma_c(acc, Qs[r * ldq + t], in[c * m2 + t]);
            out[r + c * m2] = acc;
        }
        return;
    }
    const int ncg = b / 4;                       // column groups
    for (int e = threadIdx.x; e < b * ncg; e += GT) {
        const int r = e % b, cg = e / b;
        zd acc[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = zmake(0, 0);
        const zd *q0 = Qs + r * ldq, *q1 = Qs + (r + b) * ldq;     // columns r, r+b of Q
        const zd *ic = in + (4 * cg) * m2;
        for (int t = 0; t < m2; ++t) {
            const zd a0 = q0[t], a1 = q1[t];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const zd x = ic[v * m2 + t];
                zfma_c(acc[0][v], a0, x);
                zfma_c(acc[1][v], a1, x);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            out[r + (4 * cg + v) * m2] = acc[0][v];
            out[r + b + (4 * cg + v) * m2] = acc[1][v];
        }
    }
}

// wave-wide sum (all lanes get the result)
__device__ inline zd wave_sum(zd v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    return v;
}

// Householder QR of the 2b x b window (b = 32, 256 threads) in registers: thread
// (column tid / 8, part tid % 8) holds rows part, part + 8, ... of its column.  Per
// column c the eight threads of column c form the reflector (norm and pivot entry by
// group sums) and publish it to Vh (rows above c zero) and tau to s_tau; after one
// barrier every later column takes its update.  Then Q_j = H_0 H_1 ... H_{b-1}: thread
// (column tid / 4, part tid % 4) holds rows part, part + 4, ... of a column of Q_j and
// applies the reflectors last to first, with no barrier.  On return slab holds the
// reduced window (R above, zeros below), Vh the reflectors, Ql (ld ldq) Q_j.
__device__ void ls_qr32(zd *slab, zd *Vh, double *s_tau, zd *Ql, int ldq) {
    constexpr int B = 32, M2 = 64;
    const int tid = threadIdx.x;
    {
        const int col = tid >> 3, part = tid & 7;
        zd x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = slab[(part + 8 * i) + col * M2];
#pragma unroll
        for (int c = 0; c < B; ++c) {
            if (col == c) {
                double n2 = 0.0, p0x = 0.0, p0y = 0.0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = part + 8 * i;
                    if (r >= c) n2 += zabs2(x[i]);
                    if (i == c / 8 && part == c % 8) { p0x = x[i].x; p0y = x[i].y; }
                }
                const double nrm2 = group8_sum(n2);
                const zd x0 = zmake(group8_sum(p0x), group8_sum(p0y));
                const double ax0 = sqrt(zabs2(x0)), nrm = sqrt(nrm2);
                const zd ph = (ax0 > 0.0) ? zscale(x0, 1.0 / ax0) : zmake(1.0, 0.0);
                const zd alpha = zscale(ph, -nrm);          // alpha = -phase(x0) ||x||
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = part + 8 * i;
                    const zd v = (r > c) ? x[i] : (r == c ? zsub(x[i], alpha) : zmake(0, 0));
                    Vh[r + c * M2] = v;
                    x[i] = (r == c) ? alpha : (r > c ? zmake(0, 0) : x[i]);
                }
                if (part == 0) s_tau[c] = (nrm > 0.0) ? 1.0 / (nrm * (nrm + ax0)) : 0.0;
            }
            __syncthreads();
            if (col > c) {
                zd v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = Vh[(part + 8 * i) + c * M2];
                zd d0 = zmake(0, 0), d1 = zmake(0, 0);
#pragma unroll
                for (int i = 0; i < 8; i += 2) {
                    zfma_c(d0, v[i], x[i]);
                    zfma_c(d1, v[i + 1], x[i + 1]);
                }
                const double tau = s_tau[c];
                const zd d = zscale(zmake(group8_sum(d0.x + d1.x), group8_sum(d0.y + d1.y)), tau);
#pragma unroll
                for (int i = 0; i < 8; ++i) zfms(x[i], v[i], d);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) slab[(part + 8 * i) + col * M2] = x[i];
    }
    __syncthreads();
    {
        const int qcol = tid >> 2, part = tid & 3;
        zd q[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) q[i] = zmake((part + 4 * i) == qcol ? 1.0 : 0.0, 0.0);
        for (int c = B - 1; c >= 0; --c) {                  // Q <- H_c Q
            zd v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = Vh[(part + 4 * i) + c * M2];
            zd d0 = zmake(0, 0), d1 = zmake(0, 0);
#pragma unroll
            for (int i = 0; i < 16; i += 2) {
                zfma_c(d0, v[i], q[i]);
                zfma_c(d1, v[i + 1], q[i + 1]);
            }
            const zd d = zscale(zmake(group4_sum(d0.x + d1.x), group4_sum(d0.y + d1.y)), s_tau[c]);
#pragma unroll
            for (int i = 0; i < 16; ++i) zfms(q[i], v[i], d);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Ql[(part + 4 * i) + qcol * ldq] = q[i];
    }
}

constexpr int kQPer = (64 * 64 + GT - 1) / GT;   // Q elements per thread (2b <= 64)

__global__ __launch_bounds__(GT) void ls_update_kernel(LsArgs a) {
    const int l = blockIdx.x;
    const int sb = a.active[blockIdx.y];
    const int b = a.b, j = a.j, mmax = a.mmax, nsub = a.nsub;
    const int ldc = (mmax + 1) * b;                       // column block leading dim
    const int64_t qsz = int64_t(4) * b * b;
    zd *Qs = a.Q + ls_off(l, sb, nsub, int64_t(mmax) * qsz);
    zd *R = a.R + ls_off(l, sb, nsub, int64_t(mmax) * b * mmax * b);
    const int ldr = mmax * b;
    zd *G = a.G + ls_off(l, sb, nsub, int64_t(ldc) * b);
    const zd s = a.shifts[l];
    const zd *Hc = a.H + sb * a.sH + int64_t(j) * b * a.ldh;   // block column j
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int m2 = 2 * b;
    const int ldq = m2 + 1;                               // padded: conflict-free columns

    extern __shared__ unsigned char smem_raw[];
    zd *Ql = reinterpret_cast<zd *>(smem_raw);            // [2b][2b+1]
    zd *slab = Ql + m2 * ldq;                             // [2b][b]
    zd *slab2 = slab + m2 * b;                            // [2b][b]
    zd *vv = slab2 + m2 * b;                              // [2b]

    // element (r, c) of the new column block of H - s I~ (r < (j+2) b)
    auto hval = [&](int r, int c) {
        zd v = Hc[r + int64_t(c) * a.ldh];
        if (r == j * b + c) v = zsub(v, s);
        return v;
    };
    // 1. window = rows [0, 2b)
    for (int e = tid; e < m2 * b; e += GT) {
        int r = e % m2, c = e / m2;
        slab[e] = hval(r, c);
    }
    // 2. rotations by Q_0 .. Q_{j-1}; Q_i arrives in registers one step ahead
    zd qn[kQPer];
    if (j > 0) {
#pragma unroll
        for (int q = 0; q < kQPer; ++q) {
            const int e = tid + q * GT;
            qn[q] = (e < m2 * m2) ? Qs[e] : zmake(0, 0);
        }
    }
    for (int i = 0; i < j; ++i) {
#pragma unroll
        for (int q = 0; q < kQPer; ++q) {
            const int e = tid + q * GT;
            if (e < m2 * m2) Ql[(e % m2) + (e / m2) * ldq] = qn[q];
        }
        // next rows of the column and the next Q, in flight during the product
        zd hn[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * GT;
            hn[q] = (e < b * b) ? hval((i + 2) * b + e % b, e / b) : zmake(0, 0);
        }
        if (i + 1 < j) {
            const zd *Qn = Qs + int64_t(i + 1) * qsz;
#pragma unroll
            for (int q = 0; q < kQPer; ++q) {
                const int e = tid + q * GT;
                qn[q] = (e < m2 * m2) ? Qn[e] : zmake(0, 0);
            }
        }
        __syncthreads();
        apply_qh(Ql, ldq, slab, slab2, b);
        __syncthreads();
        // top b rows are final (block row i of R); bottom b rows move up, new rows below
        for (int e = tid; e < b * b; e += GT) {
            int r = e % b, c = e / b;
            R[i * b + r + int64_t(j * b + c) * ldr] = slab2[r + c * m2];
            slab[r + c * m2] = slab2[b + r + c * m2];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * GT;
            if (e < b * b) slab[b + e % b + (e / b) * m2] = hn[q];
        }
        __syncthreads();
    }
    // 3. Householder QR of the bottom 2b x b block (in LDS).  Per column c: wave 0
    //    forms the reflector H_c = I - tau_c v_c v_c^H (v_c kept in slab2), then for
    //    every later column a group of threads takes the dot v_c^H slab(:, cc) (partial
    //    sums combined by lane shuffles) and applies the rank-one update to the same
    //    column, so one barrier separates the columns.  Q_j = H_0 H_1 ... H_{b-1} is then
    //    formed column by column, each column by its own thread group with no barrier.
    __shared__ double s_tau[32];
    zd *Vh = slab2;                                       // [2b][b] reflectors
    const int tpd = min(64, GT / b);                      // threads per trailing column
    const int dcol = tid / tpd, dpart = tid % tpd;
    if (b == 32) {
        __syncthreads();
        ls_qr32(slab, Vh, s_tau, Ql, ldq);
    } else {
    for (int c = 0; c < b; ++c) {
        if (wave == 0) {
            zd x = (lane >= c && lane < m2) ? slab[lane + c * m2] : zmake(0, 0);
            double nrm2 = wave_sum(zmake(zabs2(x), 0.0)).x;
            zd x0 = zmake(__shfl(x.x, c, 64), __shfl(x.y, c, 64));
            double ax0 = sqrt(zabs2(x0));
            double nrm = sqrt(nrm2);
            zd ph = (ax0 > 0.0) ? zscale(x0, 1.0 / ax0) : zmake(1.0, 0.0);
            zd alpha = zscale(ph, -nrm);                  // alpha = -phase(x0) ||x||
            if (lane < m2) {
                Vh[lane + c * m2] = (lane == c) ? zsub(x, alpha) : x;     // zero above c
                // column c itself becomes (alpha, 0, ..., 0) below row c
                if (lane == c) slab[lane + c * m2] = alpha;
                else if (lane > c) slab[lane + c * m2] = zmake(0, 0);
            }
            if (lane == 0) s_tau[c] = (nrm > 0.0) ? 1.0 / (nrm * (nrm + ax0)) : 0.0;  // 2 / v^H v
        }
        __syncthreads();
        const int cc = c + 1 + dcol;
        if (cc < b && dcol < GT / tpd) {
            const zd *vc = Vh + c * m2;
            zd *col = slab + cc * m2;
            zd d = zmake(0, 0);
            for (int r = c + dpart; r < m2; r += tpd) zfma_c(d, vc[r], col[r]);
            for (int off = tpd / 2; off > 0; off >>= 1) {
                d.x += __shfl_xor(d.x, off, 64);
                d.y += __shfl_xor(d.y, off, 64);
            }
            d = zscale(d, s_tau[c]);
            for (int r = c + dpart; r < m2; r += tpd) zfms(col[r], vc[r], d);
        }
        __syncthreads();
    }
    {
        const int tpq = min(64, GT / m2);                 // threads per column of Q_j
        const int qcol = tid / tpq, qpart = tid % tpq;
        if (qcol < m2) {
            zd *Qc = Ql + qcol * ldq;
            for (int r = qpart; r < m2; r += tpq) Qc[r] = (r == qcol) ? zmake(1.0, 0.0) : zmake(0, 0);
            for (int c = b - 1; c >= 0; --c) {            // Q <- H_c Q
                const zd *vc = Vh + c * m2;
                zd d = zmake(0, 0);
                for (int r = c + qpart; r < m2; r += tpq) zfma_c(d, vc[r], Qc[r]);
                for (int off = tpq / 2; off > 0; off >>= 1) {
                    d.x += __shfl_xor(d.x, off, 64);
                    d.y += __shfl_xor(d.y, off, 64);
                }
                d = zscale(d, s_tau[c]);
                for (int r = c + qpart; r < m2; r += tpq) zfms(Qc[r], vc[r], d);
            }
        }
    }
    }
    __syncthreads();
    zd *Qj = Qs + int64_t(j) * qsz;
    for (int e = tid; e < m2 * m2; e += GT) Qj[e] = Ql[(e % m2) + (e / m2) * ldq];
    // 4. diagonal block R_jj (upper triangle of the reduced window)
    for (int e = tid; e < b * b; e += GT) {
        int r = e % b, c = e / b;
        R[j * b + r + int64_t(j * b + c) * ldr] = (r <= c) ? slab[r + c * m2] : zmake(0, 0);
    }
    // 5. rotate the right-hand side rows [jb, (j+2)b) by Q_j^H
    for (int e = tid; e < m2 * b; e += GT) {
        int r = e % m2, c = e / m2;
        slab2[r + c * m2] = G[j * b + r + int64_t(c) * ldc];
    }
    __syncthreads();
    apply_qh(Ql, ldq, slab2, slab, b);
    __syncthreads();
    for (int e = tid; e < m2 * b; e += GT) {
        int r = e % m2, c = e / m2;
        G[j * b + r + int64_t(c) * ldc] = slab[r + c * m2];
    }
    // 6. residual of every column: norm of rows [(j+1)b, (j+2)b)
    for (int c = tid; c < b; c += GT) {
        double s2 = 0.0;
        for (int r = 0; r < b; ++r) s2 += zabs2(slab[b + r + c * m2]);
        double den = a.r0norm[sb * b + c];
        a.resid[(int64_t(l) * nsub + sb) * b + c] = (den > 0.0) ? sqrt(s2) / den : 0.0;
    }
}

// Back substitution R Y = G[0:mb] for every (shift, active sub-block), then
// Ycomb[sb] = sum_l c_l Y_l  is done by a second kernel in fixed shift order.
struct LsSolveArgs {
    int b, mmax, m, nq, nsub, cpw;
    const zd *R; const zd *G; zd *Y;
    const int *active;
};

// Right-looking block back substitution, columns split over blockIdx.z in groups of
// cpw (the columns of Y are independent).  The running right-hand side lives in LDS;
// once diagonal block I is solved, its contribution is removed from every row above
// it in parallel.
__global__ __launch_bounds__(GT) void ls_solve_kernel(LsSolveArgs a) {
    const int l = blockIdx.x;
    const int sb = a.active[blockIdx.y];
    const int b = a.b, mmax = a.mmax, m = a.m, cpw = a.cpw;
    const int c0 = blockIdx.z * cpw;
    const int mb = m * b;
    const int ldr = mmax * b, ldc = (mmax + 1) * b;
    const zd *R = a.R + ls_off(l, sb, a.nsub, int64_t(mmax) * b * mmax * b);
    const zd *G = a.G + ls_off(l, sb, a.nsub, int64_t(ldc) * b);
    zd *Y = a.Y + ls_off(l, sb, a.nsub, int64_t(mmax) * b * b);      // ld mmax*b
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    constexpr int nwaves = GT / 64;
    extern __shared__ unsigned char smem_raw[];
    zd *acc = reinterpret_cast<zd *>(smem_raw);           // [cpw][mb] running right-hand side
    zd *yb = acc + cpw * mb;                               // [cpw][b] solved block
    zd *D = yb + cpw * b;                                  // [b][b+1] diagonal block of R
    const int ldd = b + 1;
    __shared__ zd dinv[64];                                // 1 / D_kk
    for (int e = tid; e < mb * cpw; e += GT) {
        int r = e % mb, c = e / mb;
        acc[r + c * mb] = G[r + int64_t(c0 + c) * ldc];
    }
    for (int I = m - 1; I >= 0; --I) {
        const int r0 = I * b;
        for (int e = tid; e < b * b; e += GT) {
            int r = e % b, c = e / b;
            D[r + c * ldd] = R[r0 + r + int64_t(r0 + c) * ldr];
        }
        if (tid < b) {
            // 1 / d = conj(d) / |d|^2, all diagonal entries at once
            const zd d = R[r0 + tid + int64_t(r0 + tid) * ldr];
            const double s2 = 1.0 / zabs2(d);
            dinv[tid] = zmake(d.x * s2, -d.y * s2);
        }
        __syncthreads();
        // diagonal block: one wave per column, lane = row (b <= 64); the pivot entry of
        // step k is read out of lane k (wave-uniform) with readlane
        for (int c = wave; c < cpw; c += nwaves) {
            zd v = (lane < b) ? acc[r0 + lane + c * mb] : zmake(0, 0);
            for (int k = b - 1; k >= 0; --k) {
                const zd vk = zmake(
                    __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v.x), k),
                                     __builtin_amdgcn_readlane(__double2loint(v.x), k)),
                    __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v.y), k),
                                     __builtin_amdgcn_readlane(__double2loint(v.y), k)));
                const zd yk = zmul(vk, dinv[k]);
                if (lane == k) v = yk;
                else if (lane < k) zfms(v, D[lane + k * ldd], yk);
            }
            if (lane < b) {
                yb[lane + c * b] = v;
                Y[r0 + lane + int64_t(c0 + c) * ldr] = v;
            }
        }
        __syncthreads();
        // rows above: acc[0:r0] -= R[0:r0, block I] * yb
        for (int row = tid; row < r0; row += GT) {
            zd s[8];
            for (int c = 0; c < 8; ++c) s[c] = zmake(0, 0);
            // R entries in batches of 8, all loads of a batch issued before its use
            for (int k0 = 0; k0 < b; k0 += 8) {
                zd rv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    rv[u] = (k0 + u < b) ? R[row + int64_t(r0 + k0 + u) * ldr] : zmake(0, 0);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (k0 + u >= b) break;
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if (c < cpw) zfma(s[c], rv[u], yb[k0 + u + c * b]);
                }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < cpw) acc[row + c * mb] = zsub(acc[row + c * mb], s[c]);
        }
        __syncthreads();
    }
}

// Ycomb_sb = sum_l c_l Y_{l,sb}; with colcoef (device [nq][w]) the coefficient of
// column c of sub-block sb is colcoef[l][sb b + c] instead of cw[l].
__global__ void ls_combine_kernel(int b, int mmax, int m, int nq, int nsub, const zd *Y,
                                  const zd *cw, const zd *colcoef, int w, const int *active,
                                  int nact, zd *Ycomb) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int mb = m * b, ldr = mmax * b;
    if (e >= int64_t(mb) * b * nact) return;
    int ai = int(e / (int64_t(mb) * b));
    int64_t rem = e % (int64_t(mb) * b);
    int r = int(rem % mb), c = int(rem / mb);
    int sb = active[ai];
    zd s = zmake(0, 0);
    for (int l = 0; l < nq; ++l) {
        const zd *Yl = Y + ls_off(l, sb, nsub, int64_t(mmax) * b * b);
        const zd cl = colcoef ? colcoef[int64_t(l) * w + sb * b + c] : cw[l];
        zfma(s, cl, Yl[r + int64_t(c) * ldr]);
    }
    Ycomb[int64_t(sb) * ldr * b + r + int64_t(c) * ldr] = s;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_gemm_cn(int64_t n, int m, int k, zd alpha, const zd *A, int64_t lda,
                          int64_t sA, const zd *B, int64_t ldb, int64_t sB, zd beta, zd *C,
                          int64_t ldc, int64_t sC, int batch, zd *work, int64_t work_elems,
                          hipStream_t s, const int *map, int flags) {
    if (n <= 0 || m <= 0 || k <= 0 || batch <= 0) return hipSuccess;
    const int tn = k <= 32 ? 32 : TN;                        // tile width
    const int tm = m <= 32 ? 32 : TM;                        // tile height
    const int tiles = ((m + tm - 1) / tm) * ((k + tn - 1) / tn) * batch;
    int nchunks = int((1024 + tiles - 1) / tiles);          // aim for ~1024 workgroups
    int64_t maxch = (n + 255) / 256;
    if (nchunks > maxch) nchunks = int(maxch);
    int64_t cap = work_elems / (int64_t(m) * k * batch);
    if (nchunks > cap) nchunks = int(cap);
    if (nchunks < 1) return hipErrorInvalidValue;
    int64_t chunk = (n + nchunks - 1) / nchunks;
    chunk = ((chunk + TK - 1) / TK) * TK;
    nchunks = int((n + chunk - 1) / chunk);
    dim3 grid((m + tm - 1) / tm, (k + tn - 1) / tn, batch * nchunks);
#define RF_CN_LAUNCH(TMB_, TNB_)                                                                \
    hipLaunchKernelGGL((gemm_cn_mfma_kernel<TMB_, TNB_>), grid, dim3(GT), 0, s, n, m, k, A, lda,   \
                       sA, B, ldb, sB, work, nchunks, chunk, map, flags)
    if (tm == 32) {
        if (tn == 32) RF_CN_LAUNCH(2, 2);
        else RF_CN_LAUNCH(2, 4);
    } else {
        if (tn == 32) RF_CN_LAUNCH(4, 2);
        else RF_CN_LAUNCH(4, 4);
    }
#undef RF_CN_LAUNCH
    int64_t tot = 4 * int64_t(m) * k * batch;                 // four lanes per output
    hipLaunchKernelGGL(gemm_cn_reduce_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, m, k,
                       work, nchunks, alpha, beta, C, ldc, sC, batch, map, flags);
    return hipGetLastError();
}

hipError_t launch_gemm_nn(int64_t n, int m, int k, zd alpha, const zd *A, int64_t lda,
                          int64_t sA, const zd *B, int64_t ldb, int64_t sB, zd beta, zd *C,
                          int64_t ldc, int64_t sC, int batch, hipStream_t s, const int *map,
                          int flags) {
    if (n <= 0 || k <= 0 || batch <= 0) return hipSuccess;
    const int tn = k <= 32 ? 32 : TN;                        // tile width
    dim3 grid(unsigned((n + TM - 1) / TM), (k + tn - 1) / tn, batch);
    if (tn == 32)
        hipLaunchKernelGGL(gemm_nn_mfma_kernel<2>, grid, dim3(GT), 0, s, n, m, k, alpha, A, lda, sA,
                           B, ldb, sB, beta, C, ldc, sC, map, flags);
    else
        hipLaunchKernelGGL(gemm_nn_mfma_kernel<4>, grid, dim3(GT), 0, s, n, m, k, alpha, A, lda, sA,
                           B, ldb, sB, beta, C, ldc, sC, map, flags);
    return hipGetLastError();
}

hipError_t launch_chol_inv(int k, zd *S, int64_t sS, zd *Rout, int64_t sR, zd *Rinv,
                           int64_t sRi, int batch, int *status, double *dratio, double shift_rel,
                           hipStream_t s, const int *map, int flags) {
    if (batch <= 0) return hipSuccess;
    if (k <= 32) {
        hipLaunchKernelGGL((chol_inv_reg_kernel<32, 256>), dim3(batch), dim3(256), 0, s, k, S, sS, Rout, sR,
                           Rinv, sRi, status, dratio, shift_rel, map, flags);
    } else if (k <= 64) {
        hipLaunchKernelGGL((chol_inv_reg_kernel<64, 1024>), dim3(batch), dim3(1024), 0, s, k, S, sS, Rout, sR,
                           Rinv, sRi, status, dratio, shift_rel, map, flags);
    } else {
        if (map) return hipErrorInvalidValue;
        hipLaunchKernelGGL(chol_inv_kernel, dim3(batch), dim3(GT), 0, s, k, S, sS, Rout, sR, Rinv,
                           sRi, status, dratio, shift_rel);
    }
    return hipGetLastError();
}

hipError_t launch_add_block(int m, int k, zd alpha, const zd *A, int64_t lda, int64_t sA, zd *C,
                            int64_t ldc, int64_t sC, int batch, hipStream_t s, const int *map,
                            int flags) {
    int64_t tot = int64_t(m) * k * batch;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(add_block_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, m, k, alpha, A,
                       lda, sA, C, ldc, sC, batch, map, flags);
    return hipGetLastError();
}

hipError_t launch_copy_block(int64_t n, int ncols, const zd *src, int64_t lds, int64_t sS,
                             zd *dst, int64_t ldd, int64_t sD, int batch, hipStream_t s,
                             const int *map, int flags) {
    int64_t tot = n * ncols * batch;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_block_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, src,
                       lds, sS, dst, ldd, sD, batch, map, flags);
    return hipGetLastError();
}

hipError_t launch_copy_cols(int64_t n, int ncols, const zd *src, int64_t lds, zd *dst,
                            int64_t ldd, hipStream_t s) {
    int64_t tot = n * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_cols_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, src,
                       lds, dst, ldd);
    return hipGetLastError();
}

// d[i] = y_{pair[i]}^H (B x_i): the denominators of the first-order eigenvalue perturbation
__global__ __launch_bounds__(GT) void paired_dot_kernel(int64_t n, const zd *Y, int64_t ldy,
                                                        const int *pair, const zd *BX,
                                                        int64_t ldb, zd *d) {
    const int i = blockIdx.x;
    const zd *y = Y + int64_t(pair[i]) * ldy;
    const zd *bx = BX + int64_t(i) * ldb;
    zd acc = zmake(0, 0);
    for (int64_t r = threadIdx.x; r < n; r += GT) zfma_c(acc, y[r], bx[r]);
    __shared__ zd red[GT / 64];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        zd t = red[0];
        for (int k = 1; k < GT / 64; ++k) t = zadd(t, red[k]);
        d[i] = t;
    }
}

// One thread per row of M: for each stored entry (row, col) of the row,
// out = sum_i coef[i] conj(Y[row, pair[i]]) X[col, i].  Consecutive threads read
// consecutive rows of Y and nearby rows of X, so every i is a coalesced sweep.
__global__ void sampled_outer_kernel(int32_t n, const int32_t *rp, const int32_t *ci, int s,
                                     const zd *coef, const zd *Y, int64_t ldy, const int *pair,
                                     const zd *X, int64_t ldx, zd *out) {
    const int32_t r = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
        const int64_t col = ci[e];
        zd acc = zmake(0, 0);
        for (int i = 0; i < s; ++i) {
            zd yc = zmul(coef[i], zconj(Y[r + int64_t(pair[i]) * ldy]));
            zfma(acc, yc, X[col + int64_t(i) * ldx]);
        }
        out[e] = acc;
    }
}

hipError_t launch_paired_dots(int64_t n, int s, const zd *Y, int64_t ldy, const int *pair,
                              const zd *BX, int64_t ldb, zd *d, hipStream_t st) {
    if (s <= 0) return hipSuccess;
    hipLaunchKernelGGL(paired_dot_kernel, dim3(s), dim3(GT), 0, st, n, Y, ldy, pair, BX, ldb, d);
    return hipGetLastError();
}

hipError_t launch_sampled_outer(const DevCsr &M, int s, const zd *coef, const zd *Y, int64_t ldy,
                                const int *pair, const zd *X, int64_t ldx, zd *out,
                                hipStream_t st) {
    if (M.n == 0 || M.nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(sampled_outer_kernel, dim3((M.n + 255) / 256), dim3(256), 0, st, M.n,
                       M.rowptr, M.colind, s, coef, Y, ldy, pair, X, ldx, out);
    return hipGetLastError();
}

hipError_t launch_spmm(const DevCsr &M, int ncols, const zd *X, int64_t ldx, zd *Y, int64_t ldy,
                       hipStream_t s) {
    int64_t tot = int64_t(M.n) * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(spmm_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, int64_t(M.n), ncols,
                       M.rowptr, M.colind, M.val, X, ldx, Y, ldy);
    return hipGetLastError();
}

__global__ void sub_diag_kernel(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *Y,
                                int64_t ldy, const zd *lam, zd *Z, int64_t ldz) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    zd v = X[r + c * ldx];
    zfms(v, lam[c], Y[r + c * ldy]);
    Z[r + c * ldz] = v;
}

__global__ void add_diag_kernel(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *alpha,
                                zd *Z, int64_t ldz) {
    int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n * ncols) return;
    int64_t r = e % n, c = e / n;
    zfma(Z[r + c * ldz], alpha[c], X[r + c * ldx]);
}

hipError_t launch_sub_diag(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *Y,
                           int64_t ldy, const zd *lam, zd *Z, int64_t ldz, hipStream_t s) {
    int64_t tot = n * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(sub_diag_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, X, ldx,
                       Y, ldy, lam, Z, ldz);
    return hipGetLastError();
}

hipError_t launch_add_diag(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *alpha, zd *Z,
                           int64_t ldz, hipStream_t s) {
    int64_t tot = n * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(add_diag_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, X, ldx,
                       alpha, Z, ldz);
    return hipGetLastError();
}

hipError_t launch_axpby_cols(int64_t n, int ncols, zd alpha, const zd *X, int64_t ldx, zd beta,
                             const zd *Y, int64_t ldy, zd *Z, int64_t ldz, hipStream_t s) {
    int64_t tot = n * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(axpby_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, alpha, X,
                       ldx, beta, Y, ldy, Z, ldz);
    return hipGetLastError();
}

hipError_t launch_colnorms(int64_t n, int ncols, const zd *X, int64_t ldx, const zd *Y,
                           int64_t ldy, const zd *lam, double *out, hipStream_t s) {
    if (ncols == 0) return hipSuccess;
    hipLaunchKernelGGL(colnorm_kernel, dim3(ncols), dim3(GT), 0, s, n, X, ldx, Y, ldy, lam, out);
    return hipGetLastError();
}

hipError_t launch_inv_pos(int m, const double *src, double *dst, double other, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(inv_pos_kernel, dim3((m + 255) / 256), dim3(256), 0, s, m, src, dst, other);
    return hipGetLastError();
}

hipError_t launch_scale_cols(int64_t n, int ncols, zd *X, int64_t ldx, const double *inv,
                             hipStream_t s) {
    int64_t tot = n * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_cols_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, X,
                       ldx, inv);
    return hipGetLastError();
}

hipError_t launch_gaussian(int64_t n, int ncols, zd *X, int64_t ldx, uint64_t seed,
                           hipStream_t s) {
    int64_t tot = n * ncols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(gaussian_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, ncols, X, ldx,
                       seed);
    return hipGetLastError();
}

hipError_t launch_ls_update(const rf_plan &P, int j, const int *active, int nact, hipStream_t s) {
    if (nact == 0) return hipSuccess;
    LsArgs a;
    a.b = P.b; a.mmax = P.mmax; a.j = j; a.nq = int(P.shifts.size()); a.nsub = P.nsub;
    a.shifts = P.d_shifts;
    a.H = P.Hm; a.ldh = int64_t(P.mmax + 1) * P.b; a.sH = a.ldh * int64_t(P.mmax) * P.b;
    a.Q = P.lsQ; a.R = P.lsR; a.G = P.lsG; a.work = P.lsWork;
    a.resid = P.resid; a.r0norm = P.r0norm; a.active = active;
    const int b = P.b;
    size_t sm = (size_t(2 * b) * (2 * b + 1) + 4 * b * b + 2 * b) * sizeof(zd);
    hipLaunchKernelGGL(ls_update_kernel, dim3(a.nq, nact), dim3(GT), sm, s, a);
    return hipGetLastError();
}

hipError_t launch_ls_solve(const rf_plan &P, int m, const int *active, int nact, hipStream_t s) {
    if (nact == 0 || m == 0) return hipSuccess;
    LsSolveArgs a;
    a.b = P.b; a.mmax = P.mmax; a.m = m; a.nq = int(P.shifts.size()); a.nsub = P.nsub;
    a.R = P.lsR; a.G = P.lsG; a.Y = P.lsY; a.active = active;
    // columns per workgroup: up to 4 (more workgroups), as LDS allows
    const int mb = m * P.b;
    a.cpw = 0;
    for (int c = 4; c >= 1; c /= 2) {
        size_t sm = (size_t(c) * (mb + P.b) + size_t(P.b) * (P.b + 1)) * sizeof(zd);
        if (P.b % c == 0 && sm <= size_t(P.max_lds)) { a.cpw = c; break; }
    }
    if (a.cpw == 0) return hipErrorInvalidValue;
    size_t sm = (size_t(a.cpw) * (mb + P.b) + size_t(P.b) * (P.b + 1)) * sizeof(zd);
    hipLaunchKernelGGL(ls_solve_kernel, dim3(a.nq, nact, P.b / a.cpw), dim3(GT), sm, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t tot = int64_t(m) * P.b * P.b * nact;
    hipLaunchKernelGGL(ls_combine_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, P.b, P.mmax, m,
                       a.nq, P.nsub, P.lsY, P.d_oweights, P.colcoef_on ? P.d_colcoef : nullptr,
                       P.opts.w, active, nact, P.ycomb);
    return hipGetLastError();
}
