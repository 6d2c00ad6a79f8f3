// Gauss-Lobatto-Legendre tables for libsem (Sec. 3.2: Legendre polynomials on GLL points).
//
// Computed in long double and rounded once:
//  * nodes: the N+1 zeros of (1 - x^2) P_N'(x).  Since (1 - x^2) P_N' = N (P_{N-1} - x P_N), they
//    are the zeros of f(x) = x P_N(x) - P_{N-1}(x); Newton on f, whose derivative is
//    (N+1) P_N(x), from the Chebyshev-Lobatto points.
//  * weights: w_i = 2 / (N (N+1) P_N(x_i)^2).
//  * differentiation matrix from barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k):
//    D_ij = (lambda_j / lambda_i) / (x_i - x_j) for i != j, D_ii = -sum_{j != i} D_ij.
#include <cmath>

#include "sem_internal.h"

namespace sem {

static void legendre_pair(int N, long double x, long double* pN, long double* pNm1) {
  long double a = 1.0L, b = x;  // P_0, P_1
  if (N == 1) {
    *pN = b;
    *pNm1 = a;
    return;
  }
  for (int k = 2; k <= N; ++k) {
    long double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
    a = b;
    b = c;
  }
  *pN = b;
  *pNm1 = a;
}

void gll_tables(int N, double* xi, double* w, double* D) {
  const int P = N + 1;
  long double x[MAXP], lam[MAXP];
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < P; ++i) {
    long double t = -cosl(pi * i / N);
    if (i > 0 && i < N) {
      for (int it = 0; it < 200; ++it) {
        long double pN, pNm1;
        legendre_pair(N, t, &pN, &pNm1);
        long double dt = (t * pN - pNm1) / ((N + 1) * pN);
        t -= dt;
        if (fabsl(dt) < 1e-21L) break;
      }
    }
    x[i] = t;
  }
  x[0] = -1.0L;
  x[N] = 1.0L;
  for (int i = 0; i < P / 2; ++i) {  // exact mirror symmetry of the node set
    long double s = 0.5L * (x[N - i] - x[i]);
    x[i] = -s;
    x[N - i] = s;
  }
  if (P % 2) x[N / 2] = 0.0L;
  for (int i = 0; i < P; ++i) {
    long double pN, pNm1;
    legendre_pair(N, x[i], &pN, &pNm1);
    xi[i] = (double)x[i];
    w[i] = (double)(2.0L / ((long double)N * (N + 1) * pN * pN));
    long double pr = 1.0L;
    for (int k = 0; k < P; ++k)
      if (k != i) pr *= (x[i] - x[k]);
    lam[i] = 1.0L / pr;
  }
  for (int i = 0; i < P; ++i) {
    long double rs = 0.0L;
    for (int j = 0; j < P; ++j) {
      if (j == i) continue;
      long double v = (lam[j] / lam[i]) / (x[i] - x[j]);
      D[i * P + j] = (double)v;
      rs += v;
    }
    D[i * P + i] = (double)(-rs);
  }
}

}  // namespace sem
