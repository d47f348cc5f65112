/*
 * Oracle band LU with partial pivoting and band solves, complex FP64.
 *
 * TEST INFRASTRUCTURE ONLY: built beside the oracle and loaded by the oracle's
 * Python code; the product library never links or calls it.
 *
 * This is the "pre-factorize K_i = p_i B - A" step of Alg. composite
 * (Sec. 3.2 of Chen & Li) and the triangular solves of eq. linearsolve2,
 * written as the textbook column-by-column LU with partial pivoting on a band
 * matrix: at column j the pivot is the first entry of largest modulus among
 * rows j..j+kl, rows j and the pivot row are exchanged over the columns the
 * band reaches, the column below the diagonal is divided by the pivot and a
 * rank-one update is applied to the trailing band.  No blocking.
 *
 * Storage (column-major band with room for the pivoting fill):
 *   ldab = 2*kl + ku + 1, and matrix entry (i, j) lives at
 *   ab[(kl + ku + i - j) + j * ldab]   for  max(0, j-ku-kl) <= i <= min(n-1, j+kl).
 * The first kl rows of each column start as zero and receive the fill of U.
 * After factorization, U occupies rows 0..kl+ku (upper part, kl+ku
 * super-diagonals) and the multipliers of column j occupy rows
 * kl+ku+1 .. kl+ku+kl; ipiv[j] is the (0-based) row exchanged with row j.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>

typedef double complex zc;

#define AB(i, j) ab[(kv + (i) - (j)) + (int64_t)(j) * ldab]

/* returns 0 on success, j+1 if the pivot of column j is exactly zero */
int oracle_band_lu(int n, int kl, int ku, zc *ab, int *ipiv)
{
    const int ldab = 2 * kl + ku + 1;
    const int kv = kl + ku;
    int info = 0;
    int ju = 0; /* last column reached by U so far */
    for (int j = 0; j < n; ++j) {
        int last = j + kl < n - 1 ? j + kl : n - 1;
        int jp = j;
        double best = cabs(AB(j, j));
        for (int i = j + 1; i <= last; ++i) {
            double v = cabs(AB(i, j));
            if (v > best) { best = v; jp = i; }
        }
        ipiv[j] = jp;
        if (best == 0.0) { if (!info) info = j + 1; continue; }
        int reach = jp + ku < n - 1 ? jp + ku : n - 1;
        if (reach > ju) ju = reach;
        if (jp != j)
            for (int col = j; col <= ju; ++col) {
                zc t = AB(j, col); AB(j, col) = AB(jp, col); AB(jp, col) = t;
            }
        zc piv = AB(j, j);
        for (int i = j + 1; i <= last; ++i) AB(i, j) /= piv;
        for (int col = j + 1; col <= ju; ++col) {
            zc u = AB(j, col);
            if (u == 0.0) continue;
            for (int i = j + 1; i <= last; ++i) AB(i, col) -= AB(i, j) * u;
        }
    }
    return info;
}

/* Solve (P L U) X = Bm in place for nrhs columns of length n (leading dim ldb). */
void oracle_band_solve(int n, int kl, int ku, const zc *ab, const int *ipiv,
                       int nrhs, zc *bm, int64_t ldb)
{
    const int ldab = 2 * kl + ku + 1;
    const int kv = kl + ku;
    for (int c = 0; c < nrhs; ++c) {
        zc *b = bm + (int64_t)c * ldb;
        /* forward: interchanges and multipliers, column by column */
        for (int j = 0; j < n - 1; ++j) {
            int jp = ipiv[j];
            if (jp != j) { zc t = b[j]; b[j] = b[jp]; b[jp] = t; }
            int last = j + kl < n - 1 ? j + kl : n - 1;
            zc bj = b[j];
            for (int i = j + 1; i <= last; ++i) b[i] -= AB(i, j) * bj;
        }
        /* backward with U (kl+ku super-diagonals) */
        for (int j = n - 1; j >= 0; --j) {
            b[j] /= AB(j, j);
            zc bj = b[j];
            int first = j - kv > 0 ? j - kv : 0;
            for (int i = first; i < j; ++i) b[i] -= AB(i, j) * bj;
        }
    }
}
