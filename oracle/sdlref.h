/* FP64 CPU oracle for separable dictionary learning (2D-OMP + TMOD updates).
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
 * baseline call this library.  It shares no code with the GPU library.
 *
 * Conventions (all host pointers, FP64):
 *   signal k, pixel (i,j):   Y[k*m1*m2 + i + j*m1]        (column-major vec, Sec. I)
 *   D1 (m1 x n1), D2 (m2 x n2): column-major, atoms contiguous
 *   atom index a = i + n1*j  = column of D2 (x) D1 acting on vec X
 *   supp[k*s + t] (int32): t-th selected atom of signal k, -1 = unused slot
 *   coef[k*s + t]:         its coefficient (0 in unused slots)
 * Status codes: 0 ok, -1 invalid argument, -2 bad shape, -4 out of memory,
 * -5 singular system in a dictionary update (dictionary left unchanged).
 */
#ifndef SDLREF_H
#define SDLREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* 2D-OMP of N signals (Sec. III step 1).  mode 0: separable, correlations
 * D1^T R D2; mode 1: textbook 1D OMP on the explicit D2 (x) D1 with Householder
 * QR least squares.  p = number of contiguous shards (threads), as in
 * Algorithm 1's split of the data.  stop_rel: stop when max |corr| <= stop_rel*||Y_k||_F;
 * dep_eps: stop when the new Gram pivot <= dep_eps * G_aa.  res2 may be NULL. */
int sdlref_omp(int mode, int m1, int m2, int n1, int n2, int s, int64_t N,
               const double* Y, const double* D1, const double* D2,
               int32_t* supp, double* coef, double* res2,
               double stop_rel, double dep_eps, int p);
/* The same with the error-driven stop of the denoising experiments (Sec. IV): before each
 * step, a signal whose residual energy ||R_k||_F^2 is <= err2 takes no further atom (err2 <= 0:
 * off, identical to sdlref_omp).  The atom cap is s. */
int sdlref_omp_err(int mode, int m1, int m2, int n1, int n2, int s, int64_t N,
                   const double* Y, const double* D1, const double* D2,
                   int32_t* supp, double* coef, double* res2,
                   double stop_rel, double dep_eps, double err2, int p);

/* Dense partial sums of one TMOD half-step, by their definitions.
 * side 1 (Corollary 1): T_k = X_k D2^T;  A = sum T_k T_k^T (n1 x n1),
 *                       B = sum Y_k T_k^T (m1 x n1).
 * side 2 (Result 1): Z_k = D1 X_k; A = sum Z_k^T Z_k (n2 x n2),
 *                       B = sum Y_k^T Z_k (m2 x n2).
 * A, B column-major.  Sums are taken per shard in signal order, then over
 * shards in shard order. */
int sdlref_tmod_sums(int side, int m1, int m2, int n1, int n2, int s, int64_t N,
                     const double* Y, const double* D1, const double* D2,
                     const int32_t* supp, const double* coef, int p,
                     double* A, double* B);

/* One TMOD dictionary update (side 1: D1, side 2: D2) from fixed codes:
 * least-squares solve on the used atoms, normalisation, and rescaling of coef
 * so every product D1 X_k D2^T is unchanged.  w (n1 or n2, may be NULL)
 * receives the column norms used (1 for kept atoms). */
int sdlref_tmod_update(int side, int m1, int m2, int n1, int n2, int s, int64_t N,
                       const double* Y, double* D1, double* D2,
                       const int32_t* supp, double* coef, int p, double* w);

/* Algorithm 1: K iterations of (OMP, D1 update, OMP, D2 update), then a final
 * OMP.  schedule 1 instead uses (OMP, D2 update, D1 update) per iteration.
 * rmse_trace (K+1, may be NULL): RMSE of the OMP at the start of each
 * iteration and of the final OMP. */
int sdlref_learn(int m1, int m2, int n1, int n2, int s, int64_t N, int K, int schedule,
                 const double* Y, double* D1, double* D2,
                 int32_t* supp, double* coef, double* res2, double* rmse_trace,
                 double stop_rel, double dep_eps, int p);

/* Orthonormal variant (Remark 1; square dictionaries, n1 = m1, n2 = m2).
 * Codes: X_k = T_s(D1^T Y_k D2), the s largest-magnitude entries (ties: smaller atom), listed
 * in decreasing magnitude; res2 (may be NULL) from the explicit residual. */
int sdlref_ortho_code(int m1, int m2, int s, int64_t N, const double* Y, const double* D1,
                      const double* D2, int32_t* supp, double* coef, double* res2, int p);
/* Dictionary update by orthogonal Procrustes: side 1 replaces D1 by U V^T where
 * sum_k Y_k D2 X_k^T = U S V^T; side 2 replaces D2 likewise from sum_k Y_k^T D1 X_k.  SVD by
 * one-sided Jacobi rotations.  -5 (dictionary kept) if that sum is rank deficient. */
int sdlref_procrustes_update(int side, int m1, int m2, int s, int64_t N, const double* Y, double* D1,
                             double* D2, const int32_t* supp, const double* coef, int p);
/* Algorithm 1 with these codes and updates (K iterations, then final codes). */
int sdlref_learn_ortho(int m1, int m2, int s, int64_t N, int K, const double* Y, double* D1, double* D2,
                       int32_t* supp, double* coef, double* res2, double* rmse_trace, int p);

#ifdef __cplusplus
}
#endif
#endif
