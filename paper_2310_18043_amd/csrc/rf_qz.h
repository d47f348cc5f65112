// Host QZ of a small dense complex pencil (plain C++, no device code).
// Matrices are column-major with interleaved real and imaginary parts.
#pragma once

// phase times (ms) and sweep count of the last host_qz_eig call on this thread
struct QzStats { double qr_ms, ht_ms, qz_ms, vec_ms; int sweeps; };
extern thread_local QzStats host_qz_last_stats;

// Generalized Schur form of (A, B) (n x n) and its right eigenvectors: alpha, beta
// (n each), unit-norm eigenvectors in the columns of vr (n x n).  0 on success, -1 if
// the iteration did not converge.  A and B are not modified.
int host_qz_eig(int n, const double *A, const double *B, double *alpha, double *beta, double *vr);

// host_qz_eig for an upper triangular B when b_upper is set: the QR of step 1 is skipped
// and B's strict lower part is taken as zero.
int host_qz_eig_ex(int n, const double *A, const double *B, bool b_upper, double *alpha,
                   double *beta, double *vr);
