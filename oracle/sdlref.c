/* FP64 CPU oracle for separable dictionary learning.
 *
 * C. Rusu, P. Irofti, "Efficient and Parallel Separable Dictionary Learning",
 * arXiv:2007.03800.  This file states the method by its plain definitions:
 *
 *   - problem: minimise sum_k ||Y_k - D1 X_k D2^T||_F^2 with ||X_k||_0 <= s and
 *     unit-norm atoms (eq. (1));
 *   - sparse coding: 2D-OMP (Sec. III step 1, Sec. II), which equals OMP on
 *     the Kronecker dictionary D2 (x) D1 under column-major vec (Sec. I);
 *   - dictionary updates: Result 1 (D2) and Corollary 1 (D1), followed by
 *     column normalisation with the compensating rescaling of X;
 *   - iteration: Algorithm 1 (OMP, D1 update, OMP, D2 update);
 *   - the orthonormal variant of Remark 1: codes by hard thresholding T_s(D1^T Y_k D2),
 *     dictionaries by orthogonal Procrustes (polar factor of the update's B sum, by SVD).
 *
 * TEST INFRASTRUCTURE ONLY: plain loops, no blocking, no BLAS.  Only the tests,
 * the smoke check and the benchmark's CPU baseline use it; it shares no code
 * with the GPU library.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - argmax ties go to the smallest atom index a = i + n1*j;
 *   - OMP stops early when the largest unselected |correlation| is
 *     <= stop_rel*||Y_k||_F, or when the new atom's Gram pivot
 *     G_aa - ||w||^2 is <= dep_eps*G_aa (linear dependence);
 *   - an atom used by no code gives a zero row/column in the update's Gram
 *     matrix; the system decouples exactly, that atom is kept unchanged and the
 *     others are solved on the used set;
 *   - a zero column after the solve also keeps the old atom.
 */
#include "sdlref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_OK 0
#define REF_E_INVAL (-1)
#define REF_E_SHAPE (-2)
#define REF_E_NOMEM (-4)
#define REF_E_SINGULAR (-5)

/* a TMOD Gram sum whose Cholesky pivot falls to <= SPD_REL_TOL times its diagonal
 * entry is treated as not positive definite (numerically singular) */
#define SPD_REL_TOL 1e-12

static int check_dims(int m1, int m2, int n1, int n2, int s, int64_t N) {
  if (m1 <= 0 || m2 <= 0 || n1 <= 0 || n2 <= 0 || s <= 0 || N < 0) return REF_E_SHAPE;
  if ((int64_t)s > (int64_t)n1 * n2 || (int64_t)s > (int64_t)m1 * m2) return REF_E_SHAPE;
  return REF_OK;
}

/* shard r of p over N signals: [N*r/p, N*(r+1)/p)  (Algorithm 1, Setup) */
static int64_t shard_begin(int64_t N, int p, int r) { return (N * r) / p; }

/* ---------------------------------------------------------------- small dense algebra */

/* In-place Cholesky A = L L^T of an n x n symmetric matrix (row-major, leading
 * dimension n; lower triangle used).  Returns -1 on success, else the index of
 * the first pivot that is not larger than rel_tol times its diagonal entry.
 * pivots[k] receives the value under the square root of pivot k (may be NULL). */
static int cholesky(double* A, int n, double* pivots, double rel_tol) {
  for (int k = 0; k < n; ++k) {
    double d = A[k * n + k];
    const double diag = d;
    for (int l = 0; l < k; ++l) d -= A[k * n + l] * A[k * n + l];
    if (pivots) pivots[k] = d;
    if (!(d > rel_tol * diag)) return k;
    double lkk = sqrt(d);
    A[k * n + k] = lkk;
    for (int i = k + 1; i < n; ++i) {
      double v = A[i * n + k];
      for (int l = 0; l < k; ++l) v -= A[i * n + l] * A[k * n + l];
      A[i * n + k] = v / lkk;
    }
  }
  return -1;
}

/* Solve L L^T x = b in place (L lower, row-major n x n). */
static void chol_solve(const double* L, int n, double* x) {
  for (int i = 0; i < n; ++i) {
    double v = x[i];
    for (int l = 0; l < i; ++l) v -= L[i * n + l] * x[l];
    x[i] = v / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int l = i + 1; l < n; ++l) v -= L[l * n + i] * x[l];
    x[i] = v / L[i * n + i];
  }
}

/* ------------------------------------------------------------ separable 2D-OMP */

/* atom columns: d1_i = D1[:, i], d2_j = D2[:, j] */
static double col_dot(const double* D, int m, int a, int b) {
  double v = 0.0;
  for (int p = 0; p < m; ++p) v += D[p + m * a] * D[p + m * b];
  return v;
}

/* <d1_i d2_j^T, M>_F = d1_i^T M d2_j for an m1 x m2 column-major M */
static double bilinear(const double* D1, const double* D2, int m1, int m2, int i, int j,
                       const double* M) {
  double v = 0.0;
  for (int q = 0; q < m2; ++q) {
    double col = 0.0;
    for (int p = 0; p < m1; ++p) col += D1[p + m1 * i] * M[p + m1 * q];
    v += col * D2[q + m2 * j];
  }
  return v;
}

typedef struct {
  int m1, m2, n1, n2, s;
  double stop_rel, dep_eps;
  double err2; /* error-driven stop: ||r||_F^2 <= err2 ends the signal (off when <= 0) */
} omp_cfg;

/* Error-driven OMP (the denoising experiments, Sec. IV): no further atom once the
 * residual's energy is at or below the target. */
static int residual_small(const omp_cfg* c, const double* r, int M) {
  if (!(c->err2 > 0.0)) return 0;
  double v = 0.0;
  for (int e = 0; e < M; ++e) v += r[e] * r[e];
  return v <= c->err2;
}

/* One signal.  work: m1*m2 (r) + n1*m2 (tmp) + n1*n2 (alpha) + (s)^2 (G) + s (x) doubles,
 * plus n1*n2 bytes for the selection mask. */
static void omp_sep_one(const omp_cfg* c, const double* Y, const double* D1, const double* D2,
                        int32_t* supp, double* coef, double* res2, double* work,
                        unsigned char* selected) {
  const int m1 = c->m1, m2 = c->m2, n1 = c->n1, n2 = c->n2, s = c->s;
  const int M = m1 * m2, A = n1 * n2;
  double* r = work;
  double* tmp = r + M;
  double* alpha = tmp + n1 * m2;
  double* G = alpha + A;
  double* x = G + s * s;

  memcpy(r, Y, sizeof(double) * M);
  memset(selected, 0, (size_t)A);
  double ynorm = 0.0;
  for (int e = 0; e < M; ++e) ynorm += Y[e] * Y[e];
  ynorm = sqrt(ynorm);

  int t = 0;
  for (int step = 0; step < s; ++step) {
    if (residual_small(c, r, M)) break;
    /* correlations of the residual with every atom: alpha = D1^T r D2 */
    for (int q = 0; q < m2; ++q)
      for (int i = 0; i < n1; ++i) {
        double v = 0.0;
        for (int p = 0; p < m1; ++p) v += D1[p + m1 * i] * r[p + m1 * q];
        tmp[i + n1 * q] = v;
      }
    for (int j = 0; j < n2; ++j)
      for (int i = 0; i < n1; ++i) {
        double v = 0.0;
        for (int q = 0; q < m2; ++q) v += tmp[i + n1 * q] * D2[q + m2 * j];
        alpha[i + n1 * j] = v;
      }
    /* greedy choice among unselected atoms; ties -> smallest index */
    int best = -1;
    double bestv = -1.0;
    for (int a = 0; a < A; ++a) {
      if (selected[a]) continue;
      double v = fabs(alpha[a]);
      if (v > bestv) { bestv = v; best = a; }
    }
    if (best < 0 || bestv <= c->stop_rel * ynorm) break;

    /* Gram matrix of the support plus the candidate; entries of (D2 (x) D1)^T (D2 (x) D1)
     * are (d1_i^T d1_i')(d2_j^T d2_j'). Factor it from scratch. */
    supp[t] = best;
    const int n = t + 1;
    for (int k = 0; k < n; ++k)
      for (int l = 0; l <= k; ++l) {
        int ak = supp[k], al = supp[l];
        double g = col_dot(D1, m1, ak % n1, al % n1) * col_dot(D2, m2, ak / n1, al / n1);
        G[k * n + l] = g;
        G[l * n + k] = g;
      }
    double gaa = G[t * n + t];
    double* pivots = x; /* scratch: pivots of all rows, overwritten below */
    int fail = cholesky(G, n, pivots, 0.0);
    if (fail >= 0 && fail < t) { supp[t] = -1; break; } /* cannot happen: earlier rows passed */
    if (fail == t || pivots[t] <= c->dep_eps * gaa) { supp[t] = -1; break; }
    selected[best] = 1;
    t = n;

    /* least squares on the support: (D_S^T D_S) x = D_S^T vec Y */
    for (int k = 0; k < t; ++k) x[k] = bilinear(D1, D2, m1, m2, supp[k] % n1, supp[k] / n1, Y);
    chol_solve(G, t, x);

    /* residual r = Y - D1 X D2^T */
    memcpy(r, Y, sizeof(double) * M);
    for (int k = 0; k < t; ++k) {
      int i = supp[k] % n1, j = supp[k] / n1;
      for (int q = 0; q < m2; ++q)
        for (int p = 0; p < m1; ++p) r[p + m1 * q] -= x[k] * D1[p + m1 * i] * D2[q + m2 * j];
    }
    for (int k = 0; k < t; ++k) coef[k] = x[k];
  }
  for (int k = t; k < s; ++k) { supp[k] = -1; coef[k] = 0.0; }
  if (res2) {
    double v = 0.0;
    for (int e = 0; e < M; ++e) v += r[e] * r[e];
    *res2 = v;
  }
}

/* ----------------------------------------------------- 1D OMP on explicit D2 (x) D1 */

/* Least squares min ||y - A x|| by Householder QR of A (M x n, column-major, copied).
 * Returns R_nn^2 (square of the last diagonal entry of R) through *last_r2. */
static void householder_ls(const double* Acols, int M, int n, const double* y, double* x,
                           double* last_r2, double* work) {
  double* Q = work;          /* M x n copy, overwritten by R and reflectors */
  double* b = Q + (size_t)M * n;
  memcpy(Q, Acols, sizeof(double) * (size_t)M * n);
  memcpy(b, y, sizeof(double) * M);
  for (int k = 0; k < n; ++k) {
    double* a = Q + (size_t)M * k;
    double nrm = 0.0;
    for (int p = k; p < M; ++p) nrm += a[p] * a[p];
    nrm = sqrt(nrm);
    double alpha = a[k] > 0 ? -nrm : nrm; /* R_kk */
    /* v = a[k:] - alpha e_k, stored in place */
    double v0 = a[k] - alpha;
    double vnorm2 = v0 * v0;
    for (int p = k + 1; p < M; ++p) vnorm2 += a[p] * a[p];
    if (vnorm2 > 0.0) {
      a[k] = v0;
      /* apply H = I - 2 v v^T / (v^T v) to the remaining columns and b */
      for (int l = k + 1; l < n; ++l) {
        double* c = Q + (size_t)M * l;
        double d = 0.0;
        for (int p = k; p < M; ++p) d += a[p] * c[p];
        d = 2.0 * d / vnorm2;
        for (int p = k; p < M; ++p) c[p] -= d * a[p];
      }
      double d = 0.0;
      for (int p = k; p < M; ++p) d += a[p] * b[p];
      d = 2.0 * d / vnorm2;
      for (int p = k; p < M; ++p) b[p] -= d * a[p];
    }
    a[k] = alpha; /* keep R_kk on the diagonal (reflector tail no longer needed) */
    for (int p = k + 1; p < M; ++p) a[p] = 0.0;
  }
  /* back substitution R x = Q^T y */
  for (int i = n - 1; i >= 0; --i) {
    double v = b[i];
    for (int l = i + 1; l < n; ++l) v -= Q[(size_t)M * l + i] * x[l];
    x[i] = v / Q[(size_t)M * i + i];
  }
  double rnn = Q[(size_t)M * (n - 1) + (n - 1)];
  *last_r2 = rnn * rnn;
}

static void omp_kron_one(const omp_cfg* c, const double* Kd /* M x A */, const double* y,
                         int32_t* supp, double* coef, double* res2, double* work,
                         unsigned char* selected) {
  const int M = c->m1 * c->m2, A = c->n1 * c->n2, s = c->s;
  double* r = work;
  double* alpha = r + M;
  double* cols = alpha + A;             /* M x s */
  double* x = cols + (size_t)M * s;     /* s */
  double* qr = x + s;                   /* M*s + M */
  memcpy(r, y, sizeof(double) * M);
  memset(selected, 0, (size_t)A);
  double ynorm = 0.0;
  for (int e = 0; e < M; ++e) ynorm += y[e] * y[e];
  ynorm = sqrt(ynorm);
  int t = 0;
  for (int step = 0; step < s; ++step) {
    if (residual_small(c, r, M)) break;
    for (int a = 0; a < A; ++a) {
      double v = 0.0;
      for (int e = 0; e < M; ++e) v += Kd[(size_t)M * a + e] * r[e];
      alpha[a] = v;
    }
    int best = -1;
    double bestv = -1.0;
    for (int a = 0; a < A; ++a) {
      if (selected[a]) continue;
      double v = fabs(alpha[a]);
      if (v > bestv) { bestv = v; best = a; }
    }
    if (best < 0 || bestv <= c->stop_rel * ynorm) break;
    memcpy(cols + (size_t)M * t, Kd + (size_t)M * best, sizeof(double) * M);
    double r2, dnorm2 = 0.0;
    for (int e = 0; e < M; ++e) dnorm2 += Kd[(size_t)M * best + e] * Kd[(size_t)M * best + e];
    householder_ls(cols, M, t + 1, y, x, &r2, qr);
    if (!(r2 > c->dep_eps * dnorm2)) break;
    supp[t] = best;
    selected[best] = 1;
    ++t;
    for (int e = 0; e < M; ++e) {
      double v = y[e];
      for (int k = 0; k < t; ++k) v -= cols[(size_t)M * k + e] * x[k];
      r[e] = v;
    }
    for (int k = 0; k < t; ++k) coef[k] = x[k];
  }
  for (int k = t; k < s; ++k) { supp[k] = -1; coef[k] = 0.0; }
  if (res2) {
    double v = 0.0;
    for (int e = 0; e < M; ++e) v += r[e] * r[e];
    *res2 = v;
  }
}

int sdlref_omp(int mode, int m1, int m2, int n1, int n2, int s, int64_t N,
               const double* Y, const double* D1, const double* D2,
               int32_t* supp, double* coef, double* res2,
               double stop_rel, double dep_eps, int p) {
  return sdlref_omp_err(mode, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, res2, stop_rel, dep_eps, 0.0, p);
}

int sdlref_omp_err(int mode, int m1, int m2, int n1, int n2, int s, int64_t N,
                   const double* Y, const double* D1, const double* D2,
                   int32_t* supp, double* coef, double* res2,
                   double stop_rel, double dep_eps, double err2, int p) {
  int st = check_dims(m1, m2, n1, n2, s, N);
  if (st) return st;
  if ((N > 0 && (!Y || !supp || !coef)) || !D1 || !D2 || p <= 0 || (mode != 0 && mode != 1))
    return REF_E_INVAL;
  const int M = m1 * m2, A = n1 * n2;
  omp_cfg c = {m1, m2, n1, n2, s, stop_rel, dep_eps, err2};
  double* Kd = NULL;
  if (mode == 1) {
    /* explicit Kronecker dictionary: column a = i + n1 j is vec(d1_i d2_j^T) = d2_j (x) d1_i */
    Kd = (double*)malloc(sizeof(double) * (size_t)M * A);
    if (!Kd) return REF_E_NOMEM;
    for (int j = 0; j < n2; ++j)
      for (int i = 0; i < n1; ++i)
        for (int q = 0; q < m2; ++q)
          for (int pp = 0; pp < m1; ++pp)
            Kd[(size_t)M * (i + n1 * j) + pp + m1 * q] = D1[pp + m1 * i] * D2[q + m2 * j];
  }
  int err = 0;
#pragma omp parallel for schedule(static, 1) num_threads(p) reduction(| : err)
  for (int r = 0; r < p; ++r) {
    size_t wn = (size_t)M + (size_t)n1 * m2 + A + (size_t)s * s + s + (size_t)M * s * 2 + M + 64;
    double* work = (double*)malloc(sizeof(double) * wn);
    unsigned char* sel = (unsigned char*)malloc((size_t)A);
    if (!work || !sel) { err |= 1; free(work); free(sel); continue; }
    for (int64_t k = shard_begin(N, p, r); k < shard_begin(N, p, r + 1); ++k) {
      if (mode == 0)
        omp_sep_one(&c, Y + k * M, D1, D2, supp + k * s, coef + k * s, res2 ? res2 + k : NULL, work, sel);
      else
        omp_kron_one(&c, Kd, Y + k * M, supp + k * s, coef + k * s, res2 ? res2 + k : NULL, work, sel);
    }
    free(work);
    free(sel);
  }
  free(Kd);
  return err ? REF_E_NOMEM : REF_OK;
}

/* ------------------------------------------------------------------ TMOD sums */

/* dense X_k (n1 x n2, column-major) from its sparse code */
static void densify(int n1, int n2, int s, const int32_t* supp, const double* coef, double* X) {
  memset(X, 0, sizeof(double) * (size_t)n1 * n2);
  for (int t = 0; t < s; ++t)
    if (supp[t] >= 0) X[supp[t]] += coef[t];
}

/* Add the contribution of signal Yk with code Xk to (A, B) for the given side. */
static void add_sums(int side, int m1, int m2, int n1, int n2, const double* Yk, const double* D1,
                     const double* D2, const double* X, double* F, double* A, double* B) {
  if (side == 1) {
    /* T = X D2^T (n1 x m2);  A += T T^T;  B += Y T^T (m1 x n1) */
    for (int q = 0; q < m2; ++q)
      for (int i = 0; i < n1; ++i) {
        double v = 0.0;
        for (int j = 0; j < n2; ++j) v += X[i + n1 * j] * D2[q + m2 * j];
        F[i + n1 * q] = v;
      }
    for (int i2 = 0; i2 < n1; ++i2)
      for (int i = 0; i < n1; ++i) {
        double v = 0.0;
        for (int q = 0; q < m2; ++q) v += F[i + n1 * q] * F[i2 + n1 * q];
        A[i + n1 * i2] += v;
      }
    for (int i = 0; i < n1; ++i)
      for (int pp = 0; pp < m1; ++pp) {
        double v = 0.0;
        for (int q = 0; q < m2; ++q) v += Yk[pp + m1 * q] * F[i + n1 * q];
        B[pp + m1 * i] += v;
      }
  } else {
    /* Z = D1 X (m1 x n2);  A += Z^T Z (n2 x n2);  B += Y^T Z (m2 x n2) */
    for (int j = 0; j < n2; ++j)
      for (int pp = 0; pp < m1; ++pp) {
        double v = 0.0;
        for (int i = 0; i < n1; ++i) v += D1[pp + m1 * i] * X[i + n1 * j];
        F[pp + m1 * j] = v;
      }
    for (int j2 = 0; j2 < n2; ++j2)
      for (int j = 0; j < n2; ++j) {
        double v = 0.0;
        for (int pp = 0; pp < m1; ++pp) v += F[pp + m1 * j] * F[pp + m1 * j2];
        A[j + n2 * j2] += v;
      }
    for (int j = 0; j < n2; ++j)
      for (int q = 0; q < m2; ++q) {
        double v = 0.0;
        for (int pp = 0; pp < m1; ++pp) v += Yk[pp + m1 * q] * F[pp + m1 * j];
        B[q + m2 * j] += v;
      }
  }
}

int sdlref_tmod_sums(int side, int m1, int m2, int n1, int n2, int s, int64_t N,
                     const double* Y, const double* D1, const double* D2,
                     const int32_t* supp, const double* coef, int p,
                     double* A, double* B) {
  int st = check_dims(m1, m2, n1, n2, s, N);
  if (st) return st;
  if ((side != 1 && side != 2) || !D1 || !D2 || !A || !B || p <= 0 ||
      (N > 0 && (!Y || !supp || !coef)))
    return REF_E_INVAL;
  const int M = m1 * m2;
  const int na = side == 1 ? n1 : n2, mb = side == 1 ? m1 : m2;
  const size_t asz = (size_t)na * na, bsz = (size_t)mb * na;
  double* part = (double*)calloc((size_t)p * (asz + bsz), sizeof(double));
  if (!part) return REF_E_NOMEM;
  int err = 0;
#pragma omp parallel for schedule(static, 1) num_threads(p) reduction(| : err)
  for (int r = 0; r < p; ++r) {
    double* X = (double*)malloc(sizeof(double) * ((size_t)n1 * n2 + (size_t)(n1 + m1) * (n2 + m2)));
    if (!X) { err |= 1; continue; }
    double* F = X + (size_t)n1 * n2;
    double* Ar = part + (size_t)r * (asz + bsz);
    double* Br = Ar + asz;
    for (int64_t k = shard_begin(N, p, r); k < shard_begin(N, p, r + 1); ++k) {
      densify(n1, n2, s, supp + k * s, coef + k * s, X);
      add_sums(side, m1, m2, n1, n2, Y + k * M, D1, D2, X, F, Ar, Br);
    }
    free(X);
  }
  if (err) { free(part); return REF_E_NOMEM; }
  /* master: sum the shard partials in shard order (Algorithm 1, steps 2 and 4) */
  memset(A, 0, sizeof(double) * asz);
  memset(B, 0, sizeof(double) * bsz);
  for (int r = 0; r < p; ++r) {
    const double* Ar = part + (size_t)r * (asz + bsz);
    for (size_t e = 0; e < asz; ++e) A[e] += Ar[e];
    for (size_t e = 0; e < bsz; ++e) B[e] += Ar[asz + e];
  }
  free(part);
  return REF_OK;
}

/* ---------------------------------------------------------------- TMOD update */

int sdlref_tmod_update(int side, int m1, int m2, int n1, int n2, int s, int64_t N,
                       const double* Y, double* D1, double* D2,
                       const int32_t* supp, double* coef, int p, double* w_out) {
  const int na = side == 1 ? n1 : n2, mb = side == 1 ? m1 : m2;
  double* A = (double*)malloc(sizeof(double) * ((size_t)na * na * 2 + (size_t)mb * na * 2 + na * 2));
  if (!A) return REF_E_NOMEM;
  double* B = A + (size_t)na * na;
  double* Lm = B + (size_t)mb * na;
  double* Dn = Lm + (size_t)na * na; /* new dictionary, mb x na column-major */
  double* w = Dn + (size_t)mb * na;
  int st = sdlref_tmod_sums(side, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, p, A, B);
  if (st) { free(A); return st; }
  double* D = side == 1 ? D1 : D2;

  /* used atoms: positive diagonal of the Gram sum */
  int U[4096];
  int nu = 0;
  if (na > 4096) { free(A); return REF_E_SHAPE; }
  for (int i = 0; i < na; ++i)
    if (A[i + na * i] > 0.0) U[nu++] = i;

  /* Corollary 1 / Result 1: D* (mb x na) solves D* A = B on the used set,
   * i.e. A_UU (D*_U)^T = (B_U)^T with A_UU symmetric positive definite. */
  for (int k = 0; k < nu; ++k)
    for (int l = 0; l < nu; ++l) Lm[k * nu + l] = A[U[k] + na * U[l]];
  if (nu > 0 && cholesky(Lm, nu, NULL, SPD_REL_TOL) >= 0) { free(A); return REF_E_SINGULAR; }
  memcpy(Dn, D, sizeof(double) * (size_t)mb * na);
  double rhs[4096];
  for (int pp = 0; pp < mb; ++pp) {
    for (int k = 0; k < nu; ++k) rhs[k] = B[pp + mb * U[k]];
    chol_solve(Lm, nu, rhs);
    for (int k = 0; k < nu; ++k) Dn[pp + mb * U[k]] = rhs[k];
  }
  /* normalisation W (Result 1 / Corollary 1): unit-norm columns */
  for (int i = 0; i < na; ++i) w[i] = 1.0;
  for (int k = 0; k < nu; ++k) {
    int i = U[k];
    double nrm = 0.0;
    for (int pp = 0; pp < mb; ++pp) nrm += Dn[pp + mb * i] * Dn[pp + mb * i];
    nrm = sqrt(nrm);
    if (nrm > 0.0) {
      w[i] = nrm;
      for (int pp = 0; pp < mb; ++pp) D[pp + mb * i] = Dn[pp + mb * i] / nrm;
    }
  }
  /* X_k <- W1^{-1} X_k scaling of rows (side 1) or X_k W2^{-1} of columns (side 2),
   * with W the diagonal that normalised D*: coefficient of atom (i,j) times w */
  for (int64_t k = 0; k < N; ++k)
    for (int t = 0; t < s; ++t) {
      int32_t a = supp[k * s + t];
      if (a < 0) continue;
      int idx = side == 1 ? a % n1 : a / n1;
      coef[k * s + t] *= w[idx];
    }
  if (w_out) memcpy(w_out, w, sizeof(double) * na);
  free(A);
  return REF_OK;
}

/* ------------------------------------------------------------------ learning */

static double rmse_of(const double* res2, int64_t N, int M) {
  double v = 0.0;
  for (int64_t k = 0; k < N; ++k) v += res2[k];
  return N > 0 ? sqrt(v / ((double)N * M)) : 0.0;
}

int sdlref_learn(int m1, int m2, int n1, int n2, int s, int64_t N, int K, int schedule,
                 const double* Y, double* D1, double* D2,
                 int32_t* supp, double* coef, double* res2, double* rmse_trace,
                 double stop_rel, double dep_eps, int p) {
  int st = check_dims(m1, m2, n1, n2, s, N);
  if (st) return st;
  if (K < 0 || (schedule != 0 && schedule != 1) || !res2) return REF_E_INVAL;
  int sticky = REF_OK;
  const int M = m1 * m2;
  for (int it = 0; it < K; ++it) {
    st = sdlref_omp(0, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, res2, stop_rel, dep_eps, p);
    if (st) return st;
    if (rmse_trace) rmse_trace[it] = rmse_of(res2, N, M);
    if (schedule == 0) {
      /* Algorithm 1 steps 1-2: codes, then D1 */
      st = sdlref_tmod_update(1, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, p, NULL);
      if (st == REF_E_SINGULAR) sticky = st; else if (st) return st;
      /* steps 3-4: codes with the new D1, then D2 */
      st = sdlref_omp(0, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, res2, stop_rel, dep_eps, p);
      if (st) return st;
      st = sdlref_tmod_update(2, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, p, NULL);
      if (st == REF_E_SINGULAR) sticky = st; else if (st) return st;
    } else {
      /* Sec. III order: codes, D2, then D1 with the same (rescaled) codes */
      st = sdlref_tmod_update(2, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, p, NULL);
      if (st == REF_E_SINGULAR) sticky = st; else if (st) return st;
      st = sdlref_tmod_update(1, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, p, NULL);
      if (st == REF_E_SINGULAR) sticky = st; else if (st) return st;
    }
  }
  st = sdlref_omp(0, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, res2, stop_rel, dep_eps, p);
  if (st) return st;
  if (rmse_trace) rmse_trace[K] = rmse_of(res2, N, M);
  return sticky;
}

/* ------------------------------------------------- orthonormal variant (Remark 1) */

/* Remark 1, codes: with orthonormal D1 (m1 x m1) and D2 (m2 x m2), X_k = T_s(D1^T Y_k D2), the
 * s entries of C = D1^T Y_k D2 of largest magnitude (ties: smaller atom a = i + m1*j), listed in
 * decreasing magnitude; res2 = ||Y_k - D1 X_k D2^T||_F^2 from the explicit residual. */
int sdlref_ortho_code(int m1, int m2, int s, int64_t N, const double* Y, const double* D1,
                      const double* D2, int32_t* supp, double* coef, double* res2, int p) {
  int st = check_dims(m1, m2, m1, m2, s, N);
  if (st) return st;
  if (!D1 || !D2 || p <= 0 || (N > 0 && (!Y || !supp || !coef))) return REF_E_INVAL;
  const int M = m1 * m2;
  int err = 0;
#pragma omp parallel for schedule(static, 1) num_threads(p) reduction(| : err)
  for (int r = 0; r < p; ++r) {
    double* C = (double*)malloc(sizeof(double) * (size_t)(2 * M + m1 * m2));
    char* used = (char*)malloc((size_t)M);
    if (!C || !used) { free(C); free(used); err |= 1; continue; }
    double* R = C + M;
    for (int64_t k = shard_begin(N, p, r); k < shard_begin(N, p, r + 1); ++k) {
      const double* Yk = Y + k * M;
      for (int j = 0; j < m2; ++j)
        for (int i = 0; i < m1; ++i) C[i + m1 * j] = bilinear(D1, D2, m1, m2, i, j, Yk);
      memset(used, 0, (size_t)M);
      for (int t = 0; t < s; ++t) {
        int best = -1;
        for (int a = 0; a < M; ++a)
          if (!used[a] && (best < 0 || fabs(C[a]) > fabs(C[best]))) best = a;
        used[best] = 1;
        supp[k * s + t] = best;
        coef[k * s + t] = C[best];
      }
      if (res2) {
        memcpy(R, Yk, sizeof(double) * M);
        for (int t = 0; t < s; ++t) {
          const int a = supp[k * s + t], i = a % m1, j = a / m1;
          for (int q = 0; q < m2; ++q)
            for (int pp = 0; pp < m1; ++pp) R[pp + m1 * q] -= coef[k * s + t] * D1[pp + m1 * i] * D2[q + m2 * j];
        }
        double e = 0.0;
        for (int x = 0; x < M; ++x) e += R[x] * R[x];
        res2[k] = e;
      }
    }
    free(C);
    free(used);
  }
  return err ? REF_E_NOMEM : REF_OK;
}

/* Singular value decomposition of a square n x n matrix W (column-major, overwritten with
 * U diag(sigma)) by one-sided Jacobi rotations (Hestenes): column pairs are rotated until
 * mutually orthogonal, the rotations accumulate in V (n x n, column-major).  Returns the number
 * of sweeps, or -1 if it did not converge in 60. */
static int jacobi_svd(double* W, double* V, int n) {
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[i + n * i] = 1.0;
  for (int sweep = 1; sweep <= 60; ++sweep) {
    int rotated = 0;
    for (int i = 0; i < n - 1; ++i)
      for (int j = i + 1; j < n; ++j) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int x = 0; x < n; ++x) {
          a += W[x + n * i] * W[x + n * i];
          b += W[x + n * j] * W[x + n * j];
          g += W[x + n * i] * W[x + n * j];
        }
        if (fabs(g) <= 1e-15 * sqrt(a * b) || g == 0.0) continue;
        rotated = 1;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        for (int x = 0; x < n; ++x) {
          const double wi = W[x + n * i], wj = W[x + n * j];
          W[x + n * i] = c * wi - sn * wj;
          W[x + n * j] = sn * wi + c * wj;
          const double vi = V[x + n * i], vj = V[x + n * j];
          V[x + n * i] = c * vi - sn * vj;
          V[x + n * j] = sn * vi + c * vj;
        }
      }
    if (!rotated) return sweep;
  }
  return -1;
}

/* Remark 1, dictionary update: the orthonormal D1 minimising sum_k ||Y_k - D1 X_k D2^T||^2 for
 * fixed codes maximises tr(D1^T B1) with B1 = sum_k Y_k D2 X_k^T (the B sum of Corollary 1), so it
 * is the orthogonal Procrustes solution D1 = U V^T of B1 = U S V^T; side 2 likewise with
 * B2 = sum_k Y_k^T D1 X_k (the B sum of Result 1).  A rank-deficient B has no unique solution:
 * REF_E_SINGULAR, dictionary unchanged.  The codes are not rescaled (the atoms stay unit norm). */
int sdlref_procrustes_update(int side, int m1, int m2, int s, int64_t N, const double* Y, double* D1,
                             double* D2, const int32_t* supp, const double* coef, int p) {
  if (side != 1 && side != 2) return REF_E_INVAL;
  const int n = side == 1 ? m1 : m2;
  double* A = (double*)malloc(sizeof(double) * (size_t)n * n * 4);
  if (!A) return REF_E_NOMEM;
  double* B = A + (size_t)n * n;
  double* V = B + (size_t)n * n;
  int st = sdlref_tmod_sums(side, m1, m2, m1, m2, s, N, Y, D1, D2, supp, coef, p, A, B);
  if (st) { free(A); return st; }
  if (jacobi_svd(B, V, n) < 0) { free(A); return REF_E_SINGULAR; }
  double smax = 0.0, sig[4096];
  if (n > 4096) { free(A); return REF_E_SHAPE; }
  for (int i = 0; i < n; ++i) {
    double v = 0.0;
    for (int x = 0; x < n; ++x) v += B[x + n * i] * B[x + n * i];
    sig[i] = sqrt(v);
    if (sig[i] > smax) smax = sig[i];
  }
  for (int i = 0; i < n; ++i)
    if (!(sig[i] > 1e-12 * smax)) { free(A); return REF_E_SINGULAR; }
  double* D = side == 1 ? D1 : D2;
  /* D = U V^T with U = B V diag(1/sigma) (the columns of the rotated B, normalised) */
  for (int c = 0; c < n; ++c)
    for (int x = 0; x < n; ++x) {
      double v = 0.0;
      for (int i = 0; i < n; ++i) v += (B[x + n * i] / sig[i]) * V[c + n * i];
      D[x + n * c] = v;
    }
  free(A);
  return REF_OK;
}

/* Algorithm 1 with the orthonormal updates of Remark 1: K iterations of (T_s codes, D1 update,
 * T_s codes, D2 update), then final codes; rmse_trace[t] = RMSE of the codes at the start of
 * iteration t (t = K: the final codes). */
int sdlref_learn_ortho(int m1, int m2, int s, int64_t N, int K, const double* Y, double* D1, double* D2,
                       int32_t* supp, double* coef, double* res2, double* rmse_trace, int p) {
  int st = check_dims(m1, m2, m1, m2, s, N);
  if (st) return st;
  if (K < 0 || !res2) return REF_E_INVAL;
  int sticky = REF_OK;
  const int M = m1 * m2;
  for (int it = 0; it < K; ++it) {
    st = sdlref_ortho_code(m1, m2, s, N, Y, D1, D2, supp, coef, res2, p);
    if (st) return st;
    if (rmse_trace) rmse_trace[it] = rmse_of(res2, N, M);
    st = sdlref_procrustes_update(1, m1, m2, s, N, Y, D1, D2, supp, coef, p);
    if (st == REF_E_SINGULAR) sticky = st; else if (st) return st;
    st = sdlref_ortho_code(m1, m2, s, N, Y, D1, D2, supp, coef, res2, p);
    if (st) return st;
    st = sdlref_procrustes_update(2, m1, m2, s, N, Y, D1, D2, supp, coef, p);
    if (st == REF_E_SINGULAR) sticky = st; else if (st) return st;
  }
  st = sdlref_ortho_code(m1, m2, s, N, Y, D1, D2, supp, coef, res2, p);
  if (st) return st;
  if (rmse_trace) rmse_trace[K] = rmse_of(res2, N, M);
  return sticky;
}
