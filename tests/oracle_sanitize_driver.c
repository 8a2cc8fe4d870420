/* Runs every oracle entry point on small seeded problems; built with the address and
 * undefined-behaviour sanitizers by tests/test_oracle_sanitize.py.  Prints "ok". */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sdlref.h"

static uint64_t state = 12345u;
static double unif(void) {
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return ((double)(state >> 11) / 9007199254740992.0) * 2.0 - 1.0;
}

static void dict(double* D, int m, int n) {
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
      D[i + m * j] = unif();
      s += D[i + m * j] * D[i + m * j];
    }
    for (int i = 0; i < m; ++i) D[i + m * j] /= sqrt(s);
  }
}

static int run(int m1, int m2, int n1, int n2, int s, int64_t N) {
  const int64_t M = (int64_t)m1 * m2;
  double* Y = malloc(sizeof(double) * (size_t)(M * (N > 0 ? N : 1)));
  double* D1 = malloc(sizeof(double) * (size_t)(m1 * n1));
  double* D2 = malloc(sizeof(double) * (size_t)(m2 * n2));
  int32_t* supp = malloc(sizeof(int32_t) * (size_t)(s * (N > 0 ? N : 1)));
  double* coef = malloc(sizeof(double) * (size_t)(s * (N > 0 ? N : 1)));
  double* res2 = malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* A = malloc(sizeof(double) * (size_t)((n1 > n2 ? n1 : n2) * (n1 > n2 ? n1 : n2)));
  double* B = malloc(sizeof(double) * (size_t)((m1 > m2 ? m1 : m2) * (n1 > n2 ? n1 : n2)));
  double* w = malloc(sizeof(double) * (size_t)(n1 > n2 ? n1 : n2));
  double trace[3];
  int bad = 0;
  dict(D1, m1, n1);
  dict(D2, m2, n2);
  for (int64_t e = 0; e < M * N; ++e) Y[e] = unif();
  if (N > 1)
    for (int64_t e = 0; e < M; ++e) Y[M + e] = 0.0; /* a zero signal */
  for (int mode = 0; mode < 2; ++mode)
    bad |= sdlref_omp(mode, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, res2, 1e-14, 1e-10, 2) != 0;
  for (int mode = 0; mode < 2; ++mode) /* error-driven stop at about a third of a signal's energy */
    bad |= sdlref_omp_err(mode, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, res2, 1e-14, 1e-10, 0.1 * (double)M,
                          2) != 0;
  for (int side = 1; side <= 2; ++side) {
    bad |= sdlref_tmod_sums(side, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, 2, A, B) != 0;
    const int st = sdlref_tmod_update(side, m1, m2, n1, n2, s, N, Y, D1, D2, supp, coef, 2, w);
    bad |= st != 0 && st != -5; /* singular is a valid outcome */
  }
  for (int schedule = 0; schedule < 2; ++schedule) {
    const int st = sdlref_learn(m1, m2, n1, n2, s, N, 2, schedule, Y, D1, D2, supp, coef, res2, trace, 1e-14, 1e-10, 2);
    bad |= st != 0 && st != -5;
  }
  free(Y); free(D1); free(D2); free(supp); free(coef); free(res2); free(A); free(B); free(w);
  return bad;
}

/* the orthonormal variant (Remark 1) on square dictionaries */
static int run_ortho(int m1, int m2, int s, int64_t N) {
  const int64_t M = (int64_t)m1 * m2;
  double* Y = malloc(sizeof(double) * (size_t)(M * (N > 0 ? N : 1)));
  double* D1 = malloc(sizeof(double) * (size_t)(m1 * m1));
  double* D2 = malloc(sizeof(double) * (size_t)(m2 * m2));
  int32_t* supp = malloc(sizeof(int32_t) * (size_t)(s * (N > 0 ? N : 1)));
  double* coef = malloc(sizeof(double) * (size_t)(s * (N > 0 ? N : 1)));
  double* res2 = malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double trace[4];
  int bad = 0;
  for (int i = 0; i < m1 * m1; ++i) D1[i] = (i % (m1 + 1)) == 0 ? 1.0 : 0.0; /* identity */
  for (int i = 0; i < m2 * m2; ++i) D2[i] = (i % (m2 + 1)) == 0 ? 1.0 : 0.0;
  for (int64_t e = 0; e < M * N; ++e) Y[e] = unif();
  bad |= sdlref_ortho_code(m1, m2, s, N, Y, D1, D2, supp, coef, res2, 2) != 0;
  for (int side = 1; side <= 2; ++side) {
    const int st = sdlref_procrustes_update(side, m1, m2, s, N, Y, D1, D2, supp, coef, 2);
    bad |= st != 0 && st != -5;
  }
  const int st = sdlref_learn_ortho(m1, m2, s, N, 3, Y, D1, D2, supp, coef, res2, trace, 2);
  bad |= st != 0 && st != -5;
  free(Y); free(D1); free(D2); free(supp); free(coef); free(res2);
  return bad;
}

int main(void) {
  int bad = 0;
  bad |= run(4, 3, 5, 6, 3, 17);
  bad |= run(8, 8, 12, 12, 4, 40);
  bad |= run(3, 3, 4, 4, 1, 9);
  bad |= run(5, 4, 6, 7, 2, 0);
  bad |= run_ortho(8, 8, 8, 60);
  bad |= run_ortho(5, 3, 4, 11);
  bad |= run_ortho(4, 4, 2, 0);
  if (bad) {
    printf("bad status\n");
    return 1;
  }
  printf("ok\n");
  return 0;
}
