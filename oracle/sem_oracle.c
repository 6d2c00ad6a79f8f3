/*
 * sem_oracle.c -- plain FP64 CPU oracle for the matrix-free spectral-element
 * viscous-Burgers operators, their Jacobian products and the RK4 adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
 * binding includes, links or calls this file; only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark do.  It shares no code with
 * the HIP path.
 *
 * Everything follows Marin, Constantinescu & Smith, "A scalable matrix-free
 * spectral element approach for unsteady PDE constrained optimization using
 * PETSc/TAO" (arXiv 1806.01422):
 *   - PDE u_t = nu*Lap(u) - (u.grad)u on a periodic box        (Sec. 3, eq. burgers23d)
 *   - weak form / Galerkin SEM on GLL points                   (Sec. 3.2, eq. weakcd)
 *   - M du/dt = -nu K u - u o D u, K = D^T M D, M diagonal      (Sec. 3.2, eq. discrete1d)
 *   - affine element map, M_1=(L/2)M, K_1=(2/L)K               (Sec. 3.2)
 *   - Kronecker (sum-factorised) operators in d dimensions     (Sec. 3.3, eq. discrete3d, rhsvec)
 *   - matrix-free Jacobian J w                                 (Sec. 3.3, eq. jacvec)
 *   - matrix-free Jacobian transpose J^T w                     (Sec. 3.3, eq. jactransvec)
 *   - explicit form u' = M^{-1} P(u)                            (Sec. 3.4)
 *   - discrete adjoint of an explicit one-step method          (Sec. 4.1, eqs. adjointloop, initadj,
 *                                                                gradient, adjtime)
 *   - checkpoint-and-recompute of the forward trajectory       (Sec. 5.3, 5.4)
 *   - the three-stage explicit RK-3 of the scalability runs    (Sec. 6.3), with its adjoint
 *
 * Readings taken where the paper is silent or garbled (listed in the design notes):
 *   * Signs follow the PDE: F = -nu K u - (u.grad)u (the 1-D Jacobian formulas of Sec. 3.2 carry
 *     sign/transposition slips; the 3-D J^T of eq. jactransvec is used as the authority).
 *   * "N" is the polynomial order; an element carries N+1 GLL points per direction.
 *   * M is the GLL-collocation (lumped, diagonal) mass.  F = M^{-1} Q^T a(Q u).
 *   * J^T is the Euclidean transpose of J on unique global nodes: J^T = Q^T a'(Qu)^T Q M^{-1}.
 *   * The integrator is classical four-stage RK with a fixed step; its discrete adjoint is the
 *     reverse sweep through the four stages.
 *
 * Data layout (shared with the caller): a field is [batch][component][z][y][x], x fastest, with
 * n_d = E_d * N unique periodic nodes along direction d.  Global node g_d of element e_d, local
 * index q_d is (e_d*N + q_d) mod n_d; element e_d covers [e_d*h_d, (e_d+1)*h_d], h_d = L_d/E_d.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXP 17 /* N <= 16 */

typedef struct {
  int32_t dim;   /* 1, 2 or 3; a field has dim velocity components */
  int32_t N;     /* polynomial order */
  int32_t E[3];  /* elements per direction (unused directions ignored) */
  double L[3];   /* periodic box lengths */
  double nu;     /* viscosity */
  int32_t batch; /* independent fields stacked on the leading axis */
} orc_desc;

/* Mesh constants derived from a descriptor. */
typedef struct {
  int dim, N, P, C, batch;
  int E[3], n[3];
  double h[3], nu;
  long nodes;    /* unique nodes per component */
  long ndof;     /* nodes * C (one batch member) */
  long nelem;    /* elements */
  long nloc;     /* P^dim local nodes per element */
  double xi[ORC_MAXP], w[ORC_MAXP], D[ORC_MAXP][ORC_MAXP];
} mesh;

/* ------------------------------------------------------------------------------------------ */
/* GLL tables (Sec. 3.2: Legendre polynomials on Gauss-Lobatto-Legendre points).               */
/* Textbook definitions: xi_0=-1, xi_N=1, interior nodes are the roots of P_N'.                */
/* w_i = 2 / (N(N+1) P_N(xi_i)^2).  D_ij = l_j'(xi_i) = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)),  */
/* i != j; the diagonal is fixed by D 1 = 0 (exact differentiation of constants), which equals */
/* -N(N+1)/4, 0, ..., 0, N(N+1)/4.                                                              */
/* ------------------------------------------------------------------------------------------ */

/* Legendre P_N(x) and its first derivative by the three-term recurrence. */
static void legendre(int N, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (N == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 2; k <= N; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1; /* P_k' = P_{k-2}' + (2k-1) P_{k-1} */
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1; *dp = d1;
}

int orc_gll(int N, double* xi, double* w, double* D /* (N+1)*(N+1), row i = output node */) {
  if (N < 1 || N >= ORC_MAXP) return -1;
  const int P = N + 1;
  xi[0] = -1.0; xi[N] = 1.0;
  /* interior roots of P_N' by Newton on P_N' using P_N'' from Legendre's equation
     (1-x^2) P'' = 2x P' - N(N+1) P, started from the Chebyshev-Lobatto points */
  for (int i = 1; i < N; ++i) {
    double x = -cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(N, x, &p, &dp);
      double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    xi[i] = x;
  }
  /* symmetry of the node set: xi_{N-i} = -xi_i */
  for (int i = 0; i < P / 2; ++i) {
    double s = 0.5 * (xi[N - i] - xi[i]);
    xi[i] = -s; xi[N - i] = s;
  }
  if (P % 2 == 1) xi[N / 2] = 0.0;
  double pn[ORC_MAXP];
  for (int i = 0; i < P; ++i) {
    double dp;
    legendre(N, xi[i], &pn[i], &dp);
    w[i] = 2.0 / (N * (N + 1.0) * pn[i] * pn[i]);
  }
  for (int i = 0; i < P; ++i) {
    double rs = 0.0;
    for (int j = 0; j < P; ++j) {
      if (i == j) continue;
      double v = pn[i] / (pn[j] * (xi[i] - xi[j]));
      D[i * P + j] = v;
      rs += v;
    }
    D[i * P + i] = -rs;
  }
  return 0;
}

static int mesh_init(const orc_desc* d, mesh* m) {
  if (d->dim < 1 || d->dim > 3 || d->N < 1 || d->N >= ORC_MAXP || d->batch < 1 || !(d->nu >= 0.0))
    return -1;
  memset(m, 0, sizeof(*m));
  m->dim = d->dim; m->N = d->N; m->P = d->N + 1; m->C = d->dim; m->batch = d->batch; m->nu = d->nu;
  m->nodes = 1; m->nelem = 1; m->nloc = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < d->dim) {
      if (d->E[k] < 1 || !(d->L[k] > 0.0)) return -1;
      m->E[k] = d->E[k]; m->n[k] = d->E[k] * d->N; m->h[k] = d->L[k] / d->E[k];
    } else {
      m->E[k] = 1; m->n[k] = 1; m->h[k] = 1.0;
    }
    m->nodes *= m->n[k]; m->nelem *= m->E[k];
    if (k < d->dim) m->nloc *= m->P;
  }
  m->ndof = m->nodes * m->C;
  double Dt[ORC_MAXP * ORC_MAXP];
  if (orc_gll(m->N, m->xi, m->w, Dt)) return -1;
  for (int i = 0; i < m->P; ++i)
    for (int j = 0; j < m->P; ++j) m->D[i][j] = Dt[i * m->P + j];
  return 0;
}

/* local index q -> (q0,q1,q2); unused directions are 0 */
static void split_local(const mesh* m, long q, int qd[3]) {
  qd[0] = qd[1] = qd[2] = 0;
  for (int k = 0; k < m->dim; ++k) { qd[k] = (int)(q % m->P); q /= m->P; }
}

static void split_elem(const mesh* m, long e, int ed[3]) {
  ed[0] = (int)(e % m->E[0]); e /= m->E[0];
  ed[1] = (int)(e % m->E[1]); e /= m->E[1];
  ed[2] = (int)e;
}

/* global node of (element, local node): g_d = (e_d N + q_d) mod n_d */
static long global_node(const mesh* m, const int ed[3], const int qd[3]) {
  long g = 0, stride = 1;
  for (int k = 0; k < 3; ++k) {
    long gk = (k < m->dim) ? ((long)ed[k] * m->N + qd[k]) % m->n[k] : 0;
    g += gk * stride;
    stride *= m->n[k];
  }
  return g;
}

/* omega(q) = prod_d (h_d/2) w_{q_d}: the element's GLL quadrature weight (diagonal local mass) */
static double omega(const mesh* m, const int qd[3]) {
  double o = 1.0;
  for (int k = 0; k < m->dim; ++k) o *= 0.5 * m->h[k] * m->w[qd[k]];
  return o;
}

/* assembled diagonal mass at global node: M[g] = sum over the elements sharing g of omega,
   which for the uniform periodic mesh factorises into 1-D sums m_d(g_d). */
static double mass_at(const mesh* m, long g) {
  double M = 1.0;
  for (int k = 0; k < m->dim; ++k) {
    long gk = g % m->n[k];
    g /= m->n[k];
    int q = (int)(gk % m->N);
    double md = (q == 0) ? 2.0 * m->w[0] : m->w[q]; /* w_0 = w_N: two elements meet at q = 0 */
    M *= 0.5 * m->h[k] * md;
  }
  return M;
}

/* (D_j V)(q) = (2/h_j) sum_m D[q_j][m] V(q; q_j <- m)        transpose = 0
   (D_j^T V)(q) = (2/h_j) sum_m D[m][q_j] V(q; q_j <- m)      transpose = 1
   One direction at a time: this is the sum factorisation of Sec. 3.3 (a Kronecker factor
   D acting on direction j, identities elsewhere). */
static void deriv(const mesh* m, int j, int transpose, const double* in, double* out) {
  const int P = m->P;
  long stride = 1;
  for (int k = 0; k < j; ++k) stride *= P;
  const double s = 2.0 / m->h[j];
  for (long q = 0; q < m->nloc; ++q) {
    int qj = (int)((q / stride) % P);
    long base = q - (long)qj * stride;
    double acc = 0.0;
    for (int mm = 0; mm < P; ++mm) {
      double Dv = transpose ? m->D[mm][qj] : m->D[qj][mm];
      acc += Dv * in[base + (long)mm * stride];
    }
    out[q] = s * acc;
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Element residuals (before direct-stiffness summation).                                      */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  double* U;   /* [C][nloc] state */
  double* V;   /* [C][nloc] direction (Jv) or M^{-1}-scaled adjoint input (J^T w) */
  double* G;   /* [C][C][nloc] G_ij = D_j U_i */
  double* H;   /* [C][C][nloc] D_j V_i */
  double* T;   /* [nloc] temporary */
  double* T2;  /* [nloc] temporary */
  double* W;   /* [nloc] omega */
} work;

static int work_alloc(const mesh* m, work* w) {
  long n = m->nloc, C = m->C;
  w->U = malloc(sizeof(double) * C * n);
  w->V = malloc(sizeof(double) * C * n);
  w->G = malloc(sizeof(double) * C * C * n);
  w->H = malloc(sizeof(double) * C * C * n);
  w->T = malloc(sizeof(double) * n);
  w->T2 = malloc(sizeof(double) * n);
  w->W = malloc(sizeof(double) * n);
  if (!w->U || !w->V || !w->G || !w->H || !w->T || !w->T2 || !w->W) return -1;
  for (long q = 0; q < n; ++q) {
    int qd[3];
    split_local(m, q, qd);
    w->W[q] = omega(m, qd);
  }
  return 0;
}
static void work_free(work* w) {
  free(w->U); free(w->V); free(w->G); free(w->H); free(w->T); free(w->T2); free(w->W);
}

static void gather(const mesh* m, const double* field /* [C][nodes] */, long e, double* loc /* [C][nloc] */,
                   int scale_by_inverse_mass) {
  int ed[3], qd[3];
  split_elem(m, e, ed);
  for (long q = 0; q < m->nloc; ++q) {
    split_local(m, q, qd);
    long g = global_node(m, ed, qd);
    double s = scale_by_inverse_mass ? 1.0 / mass_at(m, g) : 1.0;
    for (int c = 0; c < m->C; ++c) loc[c * m->nloc + q] = field[c * m->nodes + g] * s;
  }
}

/* F, element part (eq. rhsvec with the signs of the PDE):
     G_ij = D_j U_i
     R_i  = - sum_j D_j^T (nu omega G_ij) - omega sum_j U_j G_ij                       */
static void elem_rhs(const mesh* m, work* w, double* R /* [C][nloc] */) {
  const long n = m->nloc;
  const int C = m->C;
  for (int i = 0; i < C; ++i)
    for (int j = 0; j < C; ++j) deriv(m, j, 0, w->U + i * n, w->G + (i * C + j) * n);
  for (int i = 0; i < C; ++i) {
    double* Ri = R + i * n;
    for (long q = 0; q < n; ++q) Ri[q] = 0.0;
    for (int j = 0; j < C; ++j) {
      const double* Gij = w->G + (i * C + j) * n;
      for (long q = 0; q < n; ++q) w->T[q] = m->nu * w->W[q] * Gij[q];
      deriv(m, j, 1, w->T, w->T2);
      for (long q = 0; q < n; ++q) Ri[q] -= w->T2[q];
    }
    for (long q = 0; q < n; ++q) {
      double adv = 0.0;
      for (int j = 0; j < C; ++j) adv += w->U[j * n + q] * w->G[(i * C + j) * n + q];
      Ri[q] -= w->W[q] * adv;
    }
  }
}

/* J(u) v, element part (eq. jacvec): linearisation of elem_rhs in direction V:
     R_i = - sum_j D_j^T (nu omega D_j V_i) - omega sum_j ( V_j G_ij + U_j D_j V_i )     */
static void elem_jac(const mesh* m, work* w, double* R) {
  const long n = m->nloc;
  const int C = m->C;
  for (int i = 0; i < C; ++i)
    for (int j = 0; j < C; ++j) {
      deriv(m, j, 0, w->U + i * n, w->G + (i * C + j) * n);
      deriv(m, j, 0, w->V + i * n, w->H + (i * C + j) * n);
    }
  for (int i = 0; i < C; ++i) {
    double* Ri = R + i * n;
    for (long q = 0; q < n; ++q) Ri[q] = 0.0;
    for (int j = 0; j < C; ++j) {
      const double* Hij = w->H + (i * C + j) * n;
      for (long q = 0; q < n; ++q) w->T[q] = m->nu * w->W[q] * Hij[q];
      deriv(m, j, 1, w->T, w->T2);
      for (long q = 0; q < n; ++q) Ri[q] -= w->T2[q];
    }
    for (long q = 0; q < n; ++q) {
      double adv = 0.0;
      for (int j = 0; j < C; ++j)
        adv += w->V[j * n + q] * w->G[(i * C + j) * n + q] + w->U[j * n + q] * w->H[(i * C + j) * n + q];
      Ri[q] -= w->W[q] * adv;
    }
  }
}

/* J(u)^T w, element part (eq. jactransvec), acting on Z = (M^{-1} w) gathered to the element:
     R_l = - sum_j D_j^T [ omega (nu D_j Z_l + U_j Z_l) ] - omega sum_i Z_i D_l U_i        */
static void elem_jact(const mesh* m, work* w, double* R) {
  const long n = m->nloc;
  const int C = m->C;
  const double* Z = w->V;
  for (int i = 0; i < C; ++i)
    for (int j = 0; j < C; ++j) deriv(m, j, 0, w->U + i * n, w->G + (i * C + j) * n);
  for (int l = 0; l < C; ++l) {
    double* Rl = R + l * n;
    for (long q = 0; q < n; ++q) Rl[q] = 0.0;
    for (int j = 0; j < C; ++j) {
      deriv(m, j, 0, Z + l * n, w->T2); /* D_j Z_l */
      for (long q = 0; q < n; ++q) w->T[q] = w->W[q] * (m->nu * w->T2[q] + w->U[j * n + q] * Z[l * n + q]);
      deriv(m, j, 1, w->T, w->T2);
      for (long q = 0; q < n; ++q) Rl[q] -= w->T2[q];
    }
    for (long q = 0; q < n; ++q) {
      double s = 0.0;
      for (int i = 0; i < C; ++i) s += Z[i * n + q] * w->G[(i * C + l) * n + q];
      Rl[q] -= w->W[q] * s;
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Direct-stiffness summation Q^T: sum the element contributions at every shared global node,  */
/* in a fixed order so the threaded result equals the serial one.                              */
/* ------------------------------------------------------------------------------------------ */
static void assemble(const mesh* m, const double* Lvec /* [nelem][C][nloc] */, double* out /* [C][nodes] */,
                     int divide_by_mass) {
  const int dim = m->dim, N = m->N, P = m->P;
#pragma omp parallel for schedule(static)
  for (long g = 0; g < m->nodes; ++g) {
    int gd[3] = {0, 0, 0};
    long t = g;
    for (int k = 0; k < 3; ++k) { gd[k] = (int)(t % m->n[k]); t /= m->n[k]; }
    /* contributors along direction k: (element, local) pairs */
    int ne[3], ee[3][2], qq[3][2];
    for (int k = 0; k < 3; ++k) {
      if (k >= dim) { ne[k] = 1; ee[k][0] = 0; qq[k][0] = 0; continue; }
      int e0 = gd[k] / N, q0 = gd[k] % N;
      ee[k][0] = e0; qq[k][0] = q0; ne[k] = 1;
      if (q0 == 0) { ee[k][1] = (e0 - 1 + m->E[k]) % m->E[k]; qq[k][1] = N; ne[k] = 2; }
    }
    double M = divide_by_mass ? mass_at(m, g) : 1.0;
    for (int c = 0; c < m->C; ++c) {
      double s = 0.0;
      for (int a = 0; a < ne[0]; ++a)
        for (int b = 0; b < ne[1]; ++b)
          for (int cz = 0; cz < ne[2]; ++cz) {
            long e = ee[0][a] + (long)m->E[0] * (ee[1][b] + (long)m->E[1] * ee[2][cz]);
            long q = qq[0][a];
            if (dim > 1) q += (long)P * qq[1][b];
            if (dim > 2) q += (long)P * P * qq[2][cz];
            s += Lvec[(e * m->C + c) * m->nloc + q];
          }
      out[c * m->nodes + g] = s / M;
    }
  }
}

enum { OP_RHS = 0, OP_JAC = 1, OP_JACT = 2 };

/* Apply one operator to one batch member.  Lvec has nelem*C*nloc entries. */
static int apply_one(const mesh* m, int op, const double* u, const double* v, double* out, double* Lvec) {
  int fail = 0;
#pragma omp parallel reduction(| : fail)
  {
    work w;
    if (work_alloc(m, &w)) {
      fail = 1;
    } else {
#pragma omp for schedule(static)
      for (long e = 0; e < m->nelem; ++e) {
        double* R = Lvec + e * m->C * m->nloc;
        gather(m, u, e, w.U, 0);
        if (op == OP_RHS) {
          elem_rhs(m, &w, R);
        } else if (op == OP_JAC) {
          gather(m, v, e, w.V, 0);
          elem_jac(m, &w, R);
        } else {
          gather(m, v, e, w.V, 1); /* Z = M^{-1} w gathered to the element */
          elem_jact(m, &w, R);
        }
      }
    }
    work_free(&w);
  }
  if (fail) return -2;
  /* F and J v: u' = M^{-1} Q^T (...);  J^T w: no division (M^{-1} was applied to the input) */
  assemble(m, Lvec, out, op != OP_JACT);
  return 0;
}

static int apply_op(const orc_desc* d, int op, const double* u, const double* v, double* out) {
  mesh m;
  if (mesh_init(d, &m)) return -1;
  double* Lvec = malloc(sizeof(double) * m.nelem * m.C * m.nloc);
  if (!Lvec) return -2;
  int rc = 0;
  for (int b = 0; b < m.batch && !rc; ++b)
    rc = apply_one(&m, op, u + b * m.ndof, v ? v + b * m.ndof : NULL, out + b * m.ndof, Lvec);
  free(Lvec);
  return rc;
}

int orc_rhs(const orc_desc* d, const double* u, double* f) { return apply_op(d, OP_RHS, u, NULL, f); }
int orc_jac_vec(const orc_desc* d, const double* u, const double* v, double* jv) {
  return apply_op(d, OP_JAC, u, v, jv);
}
int orc_jact_vec(const orc_desc* d, const double* u, const double* w, double* jtw) {
  return apply_op(d, OP_JACT, u, w, jtw);
}

/* ------------------------------------------------------------------------------------------ */
/* Time integration: classical RK4 on u' = F(u) with a fixed step, its tangent-linear model    */
/* and its discrete adjoint (Sec. 4.1: the adjoint of the one-step map, applied in reverse).    */
/* All vectors here are one batch member (ndof entries).                                        */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  mesh m;
  double* Lvec;
  double *k1, *k2, *k3, *k4, *U2, *U3, *U4, *a, *t;
} stepper;

static int stepper_init(const orc_desc* d, stepper* s) {
  memset(s, 0, sizeof(*s));
  if (mesh_init(d, &s->m)) return -1;
  long n = s->m.ndof;
  s->Lvec = malloc(sizeof(double) * s->m.nelem * s->m.C * s->m.nloc);
  double** v[] = {&s->k1, &s->k2, &s->k3, &s->k4, &s->U2, &s->U3, &s->U4, &s->a, &s->t};
  for (unsigned i = 0; i < sizeof(v) / sizeof(v[0]); ++i) *v[i] = malloc(sizeof(double) * n);
  if (!s->Lvec || !s->k1 || !s->k2 || !s->k3 || !s->k4 || !s->U2 || !s->U3 || !s->U4 || !s->a || !s->t)
    return -2;
  return 0;
}
static void stepper_free(stepper* s) {
  free(s->Lvec); free(s->k1); free(s->k2); free(s->k3); free(s->k4);
  free(s->U2); free(s->U3); free(s->U4); free(s->a); free(s->t);
}

static void axpy_to(long n, double* y, const double* x0, double a, const double* x) {
  for (long i = 0; i < n; ++i) y[i] = x0[i] + a * x[i];
}

/* the four stages of one step from u: fills k1..k4 and U2..U4 */
static int rk4_stages(stepper* s, double dt, const double* u) {
  const mesh* m = &s->m;
  long n = m->ndof;
  int rc = 0;
  rc |= apply_one(m, OP_RHS, u, NULL, s->k1, s->Lvec);
  axpy_to(n, s->U2, u, 0.5 * dt, s->k1);
  rc |= apply_one(m, OP_RHS, s->U2, NULL, s->k2, s->Lvec);
  axpy_to(n, s->U3, u, 0.5 * dt, s->k2);
  rc |= apply_one(m, OP_RHS, s->U3, NULL, s->k3, s->Lvec);
  axpy_to(n, s->U4, u, dt, s->k3);
  rc |= apply_one(m, OP_RHS, s->U4, NULL, s->k4, s->Lvec);
  return rc;
}

/* u <- u + dt/6 (k1 + 2 k2 + 2 k3 + k4) */
static int rk4_step(stepper* s, double dt, double* u) {
  if (rk4_stages(s, dt, u)) return -2;
  for (long i = 0; i < s->m.ndof; ++i)
    u[i] += dt / 6.0 * (s->k1[i] + 2.0 * s->k2[i] + 2.0 * s->k3[i] + s->k4[i]);
  return 0;
}

/* Reverse sweep through one RK4 step taken from u (adjoint of the one-step map):
     a4 = J(U4)^T (dt/6 lam)
     a3 = J(U3)^T (dt/3 lam + dt   a4)
     a2 = J(U2)^T (dt/3 lam + dt/2 a3)
     a1 = J(u )^T (dt/6 lam + dt/2 a2)
     lam <- lam + a1 + a2 + a3 + a4                                                 */
static int rk4_adjoint_step(stepper* s, double dt, const double* u, double* lam) {
  const mesh* m = &s->m;
  long n = m->ndof;
  double *a1 = s->k1, *a2 = s->k2, *a3 = s->k3, *a4 = s->k4, *t = s->t;
  int rc = 0;
  if (rk4_stages(s, dt, u)) return -2; /* recompute the stage states U2..U4 */
  for (long i = 0; i < n; ++i) t[i] = dt / 6.0 * lam[i];
  rc |= apply_one(m, OP_JACT, s->U4, t, a4, s->Lvec);
  for (long i = 0; i < n; ++i) t[i] = dt / 3.0 * lam[i] + dt * a4[i];
  rc |= apply_one(m, OP_JACT, s->U3, t, a3, s->Lvec);
  for (long i = 0; i < n; ++i) t[i] = dt / 3.0 * lam[i] + 0.5 * dt * a3[i];
  rc |= apply_one(m, OP_JACT, s->U2, t, a2, s->Lvec);
  for (long i = 0; i < n; ++i) t[i] = dt / 6.0 * lam[i] + 0.5 * dt * a2[i];
  rc |= apply_one(m, OP_JACT, u, t, a1, s->Lvec);
  for (long i = 0; i < n; ++i) lam[i] += a1[i] + a2[i] + a3[i] + a4[i];
  return rc;
}

/* Tangent-linear RK4 step (forward derivative of the one-step map in direction du):
     dk1 = J(u) du;  dk2 = J(U2)(du + dt/2 dk1);  dk3 = J(U3)(du + dt/2 dk2);
     dk4 = J(U4)(du + dt dk3);  du <- du + dt/6 (dk1 + 2 dk2 + 2 dk3 + dk4);  u advances.     */
static int rk4_tlm_step(stepper* s, double dt, double* u, double* du) {
  const mesh* m = &s->m;
  long n = m->ndof;
  int rc = 0;
  if (rk4_stages(s, dt, u)) return -2;
  double *t = s->t, *dk = s->a;
  double* acc = malloc(sizeof(double) * n);
  if (!acc) return -2;
  rc |= apply_one(m, OP_JAC, u, du, dk, s->Lvec);
  for (long i = 0; i < n; ++i) { acc[i] = dk[i]; t[i] = du[i] + 0.5 * dt * dk[i]; }
  rc |= apply_one(m, OP_JAC, s->U2, t, dk, s->Lvec);
  for (long i = 0; i < n; ++i) { acc[i] += 2.0 * dk[i]; t[i] = du[i] + 0.5 * dt * dk[i]; }
  rc |= apply_one(m, OP_JAC, s->U3, t, dk, s->Lvec);
  for (long i = 0; i < n; ++i) { acc[i] += 2.0 * dk[i]; t[i] = du[i] + dt * dk[i]; }
  rc |= apply_one(m, OP_JAC, s->U4, t, dk, s->Lvec);
  for (long i = 0; i < n; ++i) {
    acc[i] += dk[i];
    du[i] += dt / 6.0 * acc[i];
    u[i] += dt / 6.0 * (s->k1[i] + 2.0 * s->k2[i] + 2.0 * s->k3[i] + s->k4[i]);
  }
  free(acc);
  return rc;
}

/* Forward trajectory of every batch member; when ckpt is non-NULL, u_{sK} is stored in
   ckpt[s][batch][ndof] for s = 0 .. nsteps/K - 1 before step sK is taken. */
int orc_rk4_forward(const orc_desc* d, double dt, int32_t nsteps, int32_t K, double* u, double* ckpt) {
  if (nsteps < 0 || (ckpt && (K < 1 || nsteps % K))) return -1;
  stepper s;
  int rc = stepper_init(d, &s);
  if (rc) { stepper_free(&s); return rc; }
  const long n = s.m.ndof, B = s.m.batch;
  for (long b = 0; b < B && !rc; ++b) {
    double* ub = u + b * n;
    for (int k = 0; k < nsteps && !rc; ++k) {
      if (ckpt && k % K == 0) memcpy(ckpt + ((long)(k / K) * B + b) * n, ub, sizeof(double) * n);
      rc = rk4_step(&s, dt, ub);
    }
  }
  stepper_free(&s);
  return rc;
}

/* Discrete adjoint with uniform checkpoints: for each segment, last to first, recompute the K
   states of the segment from its checkpoint, then sweep the K steps in reverse.  lam holds
   lambda_N on entry (per batch member) and lambda_0 = dPhi/du_0 on exit (Sec. 4.1, eq. gradient). */
int orc_rk4_adjoint(const orc_desc* d, double dt, int32_t nsteps, int32_t K, const double* ckpt, double* lam) {
  if (nsteps < 0 || K < 1 || nsteps % K) return -1;
  stepper s;
  int rc = stepper_init(d, &s);
  if (rc) { stepper_free(&s); return rc; }
  const long n = s.m.ndof, B = s.m.batch;
  double* seg = malloc(sizeof(double) * n * (size_t)K);
  if (!seg) { stepper_free(&s); return -2; }
  const int S = nsteps / K;
  for (long b = 0; b < B && !rc; ++b) {
    double* lb = lam + b * n;
    for (int sg = S - 1; sg >= 0 && !rc; --sg) {
      memcpy(seg, ckpt + ((long)sg * B + b) * n, sizeof(double) * n);
      for (int k = 1; k < K && !rc; ++k) {
        memcpy(seg + k * n, seg + (k - 1) * n, sizeof(double) * n);
        rc = rk4_step(&s, dt, seg + k * n);
      }
      for (int k = K - 1; k >= 0 && !rc; --k) rc = rk4_adjoint_step(&s, dt, seg + k * n, lb);
    }
  }
  free(seg);
  stepper_free(&s);
  return rc;
}

/* Tangent-linear trajectory: u and du advance together over nsteps (per batch member). */
int orc_rk4_tlm(const orc_desc* d, double dt, int32_t nsteps, double* u, double* du) {
  if (nsteps < 0) return -1;
  stepper s;
  int rc = stepper_init(d, &s);
  if (rc) { stepper_free(&s); return rc; }
  const long n = s.m.ndof;
  for (long b = 0; b < s.m.batch && !rc; ++b)
    for (int k = 0; k < nsteps && !rc; ++k) rc = rk4_tlm_step(&s, dt, u + b * n, du + b * n);
  stepper_free(&s);
  return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* General explicit Runge-Kutta method given by its Butcher tableau (A strictly lower          */
/* triangular, weights b): stage states U_i = u + dt sum_{j<i} A_ij k_j, k_i = F(U_i),           */
/* u+ = u + dt sum_i b_i k_i.  The discrete adjoint of that one-step map (Sec. 4.1, applied to  */
/* a general tableau) runs the stages in reverse:                                               */
/*     a_i = J(U_i)^T [ dt (b_i lam + sum_{j>i} A_ji a_j) ],   lam <- lam + sum_i a_i,           */
/* and the tangent-linear map is dk_i = J(U_i)(du + dt sum_{j<i} A_ij dk_j),                     */
/* du <- du + dt sum_i b_i dk_i.  The paper integrates with a three-stage explicit RK-3 (Sec. 6.3) */
/* without printing its tableau; scheme 1 takes Kutta's third-order method.  Scheme 0 is the    */
/* classical RK4 tableau, an independent route to the hand-written RK4 above.                   */
/* ------------------------------------------------------------------------------------------ */
#define ERK_MAXS 4
typedef struct {
  int s;
  double A[ERK_MAXS][ERK_MAXS];
  double b[ERK_MAXS];
} tableau;

static int erk_tableau(int scheme, tableau* t) {
  memset(t, 0, sizeof(*t));
  if (scheme == 0) { /* classical RK4 */
    t->s = 4;
    t->A[1][0] = 0.5;
    t->A[2][1] = 0.5;
    t->A[3][2] = 1.0;
    t->b[0] = 1.0 / 6; t->b[1] = 1.0 / 3; t->b[2] = 1.0 / 3; t->b[3] = 1.0 / 6;
    return 0;
  }
  if (scheme == 1) { /* Kutta's third-order method */
    t->s = 3;
    t->A[1][0] = 0.5;
    t->A[2][0] = -1.0; t->A[2][1] = 2.0;
    t->b[0] = 1.0 / 6; t->b[1] = 2.0 / 3; t->b[2] = 1.0 / 6;
    return 0;
  }
  return -1;
}

/* host copy of a scheme's tableau: A row-major s x s, b[s]; returns s, or -1 */
int orc_erk_tableau(int32_t scheme, double* A, double* b) {
  tableau t;
  if (erk_tableau(scheme, &t)) return -1;
  for (int i = 0; i < t.s; ++i) {
    b[i] = t.b[i];
    for (int j = 0; j < t.s; ++j) A[i * t.s + j] = t.A[i][j];
  }
  return t.s;
}

typedef struct {
  mesh m;
  tableau t;
  double* Lvec;
  double *U[ERK_MAXS], *k[ERK_MAXS], *a[ERK_MAXS], *tmp;
} erk;

static int erk_init(const orc_desc* d, int scheme, erk* r) {
  memset(r, 0, sizeof(*r));
  if (erk_tableau(scheme, &r->t)) return -1;
  if (mesh_init(d, &r->m)) return -1;
  const long n = r->m.ndof;
  r->Lvec = malloc(sizeof(double) * r->m.nelem * r->m.C * r->m.nloc);
  r->tmp = malloc(sizeof(double) * n);
  if (!r->Lvec || !r->tmp) return -2;
  for (int i = 0; i < r->t.s; ++i) {
    r->U[i] = malloc(sizeof(double) * n);
    r->k[i] = malloc(sizeof(double) * n);
    r->a[i] = malloc(sizeof(double) * n);
    if (!r->U[i] || !r->k[i] || !r->a[i]) return -2;
  }
  return 0;
}
static void erk_free(erk* r) {
  free(r->Lvec); free(r->tmp);
  for (int i = 0; i < ERK_MAXS; ++i) { free(r->U[i]); free(r->k[i]); free(r->a[i]); }
}

/* stage states U_i and stage slopes k_i of one step from u */
static int erk_stages(erk* r, double dt, const double* u) {
  const long n = r->m.ndof;
  int rc = 0;
  for (int i = 0; i < r->t.s; ++i) {
    for (long g = 0; g < n; ++g) {
      double acc = 0.0;
      for (int j = 0; j < i; ++j) acc += r->t.A[i][j] * r->k[j][g];
      r->U[i][g] = u[g] + dt * acc;
    }
    rc |= apply_one(&r->m, OP_RHS, r->U[i], NULL, r->k[i], r->Lvec);
  }
  return rc;
}

static int erk_step(erk* r, double dt, double* u) {
  if (erk_stages(r, dt, u)) return -2;
  for (long g = 0; g < r->m.ndof; ++g) {
    double acc = 0.0;
    for (int i = 0; i < r->t.s; ++i) acc += r->t.b[i] * r->k[i][g];
    u[g] += dt * acc;
  }
  return 0;
}

static int erk_adjoint_step(erk* r, double dt, const double* u, double* lam) {
  const long n = r->m.ndof;
  int rc = 0;
  if (erk_stages(r, dt, u)) return -2;
  for (int i = r->t.s - 1; i >= 0; --i) {
    for (long g = 0; g < n; ++g) {
      double acc = r->t.b[i] * lam[g];
      for (int j = i + 1; j < r->t.s; ++j) acc += r->t.A[j][i] * r->a[j][g];
      r->tmp[g] = dt * acc;
    }
    rc |= apply_one(&r->m, OP_JACT, r->U[i], r->tmp, r->a[i], r->Lvec);
  }
  for (long g = 0; g < n; ++g)
    for (int i = 0; i < r->t.s; ++i) lam[g] += r->a[i][g];
  return rc;
}

static int erk_tlm_step(erk* r, double dt, double* u, double* du) {
  const long n = r->m.ndof;
  int rc = 0;
  if (erk_stages(r, dt, u)) return -2;
  double** dk = r->a; /* reused as the stage derivatives */
  for (int i = 0; i < r->t.s; ++i) {
    for (long g = 0; g < n; ++g) {
      double acc = 0.0;
      for (int j = 0; j < i; ++j) acc += r->t.A[i][j] * dk[j][g];
      r->tmp[g] = du[g] + dt * acc;
    }
    rc |= apply_one(&r->m, OP_JAC, r->U[i], r->tmp, dk[i], r->Lvec);
  }
  for (long g = 0; g < n; ++g) {
    double acc = 0.0, accu = 0.0;
    for (int i = 0; i < r->t.s; ++i) {
      acc += r->t.b[i] * dk[i][g];
      accu += r->t.b[i] * r->k[i][g];
    }
    du[g] += dt * acc;
    u[g] += dt * accu;
  }
  return rc;
}

/* Forward trajectory with checkpoints, as orc_rk4_forward, for any tableau. */
int orc_erk_forward(const orc_desc* d, int32_t scheme, double dt, int32_t nsteps, int32_t K, double* u,
                    double* ckpt) {
  if (nsteps < 0 || (ckpt && (K < 1 || nsteps % K))) return -1;
  erk r;
  int rc = erk_init(d, scheme, &r);
  if (rc) { erk_free(&r); return rc; }
  const long n = r.m.ndof, B = r.m.batch;
  for (long b = 0; b < B && !rc; ++b) {
    double* ub = u + b * n;
    for (int k = 0; k < nsteps && !rc; ++k) {
      if (ckpt && k % K == 0) memcpy(ckpt + ((long)(k / K) * B + b) * n, ub, sizeof(double) * n);
      rc = erk_step(&r, dt, ub);
    }
  }
  erk_free(&r);
  return rc;
}

/* Discrete adjoint with uniform checkpoints and segment recompute, as orc_rk4_adjoint. */
int orc_erk_adjoint(const orc_desc* d, int32_t scheme, double dt, int32_t nsteps, int32_t K, const double* ckpt,
                    double* lam) {
  if (nsteps < 0 || K < 1 || nsteps % K) return -1;
  erk r;
  int rc = erk_init(d, scheme, &r);
  if (rc) { erk_free(&r); return rc; }
  const long n = r.m.ndof, B = r.m.batch;
  double* seg = malloc(sizeof(double) * n * (size_t)K);
  if (!seg) { erk_free(&r); return -2; }
  for (long b = 0; b < B && !rc; ++b) {
    double* lb = lam + b * n;
    for (int sg = nsteps / K - 1; sg >= 0 && !rc; --sg) {
      memcpy(seg, ckpt + ((long)sg * B + b) * n, sizeof(double) * n);
      for (int k = 1; k < K && !rc; ++k) {
        memcpy(seg + k * n, seg + (k - 1) * n, sizeof(double) * n);
        rc = erk_step(&r, dt, seg + k * n);
      }
      for (int k = K - 1; k >= 0 && !rc; --k) rc = erk_adjoint_step(&r, dt, seg + k * n, lb);
    }
  }
  free(seg);
  erk_free(&r);
  return rc;
}

/* Tangent-linear trajectory for any tableau. */
int orc_erk_tlm(const orc_desc* d, int32_t scheme, double dt, int32_t nsteps, double* u, double* du) {
  if (nsteps < 0) return -1;
  erk r;
  int rc = erk_init(d, scheme, &r);
  if (rc) { erk_free(&r); return rc; }
  const long n = r.m.ndof;
  for (long b = 0; b < r.m.batch && !rc; ++b)
    for (int k = 0; k < nsteps && !rc; ++k) rc = erk_tlm_step(&r, dt, u + b * n, du + b * n);
  erk_free(&r);
  return rc;
}

/* Misfit Phi = 1/2 sum (u - u*)^2 over all unique nodes and components (per batch member, into
   phi[b]), and its gradient with respect to u(T): lam = u - u*  (Sec. 4.1, eq. initadj, in the
   Euclidean form). */
int orc_misfit(const orc_desc* d, const double* uT, const double* utarget, double* phi, double* lam) {
  mesh m;
  if (mesh_init(d, &m)) return -1;
  for (long b = 0; b < m.batch; ++b) {
    double s = 0.0;
    for (long i = 0; i < m.ndof; ++i) {
      double r = uT[b * m.ndof + i] - utarget[b * m.ndof + i];
      if (lam) lam[b * m.ndof + i] = r;
      s += r * r;
    }
    phi[b] = 0.5 * s;
  }
  return 0;
}

/* L2 projection of an element-local (discontinuous) field onto the continuous space with the
   lumped GLL mass: out = M^{-1} Q^T (omega o loc).  loc is [batch][nelem][C][nloc]. */
int orc_project_local(const orc_desc* d, const double* loc, double* out) {
  mesh m;
  if (mesh_init(d, &m)) return -1;
  double* Lvec = malloc(sizeof(double) * m.nelem * m.C * m.nloc);
  if (!Lvec) return -2;
  for (long b = 0; b < m.batch; ++b) {
    const double* lb = loc + b * m.nelem * m.C * m.nloc;
    for (long e = 0; e < m.nelem; ++e)
      for (int c = 0; c < m.C; ++c)
        for (long q = 0; q < m.nloc; ++q) {
          int qd[3];
          split_local(&m, q, qd);
          long i = (e * m.C + c) * m.nloc + q;
          Lvec[i] = omega(&m, qd) * lb[i];
        }
    assemble(&m, Lvec, out + b * m.ndof, 1);
  }
  free(Lvec);
  return 0;
}

/* 1-D node coordinates of direction k: x_g = (g div N) h + (xi_{g mod N} + 1) h / 2 */
int orc_coords(const orc_desc* d, int32_t k, double* x) {
  mesh m;
  if (mesh_init(d, &m) || k < 0 || k >= m.dim) return -1;
  for (long g = 0; g < m.n[k]; ++g) x[g] = (g / m.N) * m.h[k] + 0.5 * (m.xi[g % m.N] + 1.0) * m.h[k];
  return 0;
}

/* assembled diagonal mass of one component: M[g] */
int orc_mass(const orc_desc* d, double* M) {
  mesh m;
  if (mesh_init(d, &m)) return -1;
  for (long g = 0; g < m.nodes; ++g) M[g] = mass_at(&m, g);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of later parallel regions (n < 1: all).  Results do not depend on it: every summation
   runs in a fixed order. */
void orc_set_threads(int n) {
#ifdef _OPENMP
  static int all = 0;
  if (!all) all = omp_get_max_threads();
  omp_set_num_threads(n >= 1 ? n : all);
#else
  (void)n;
#endif
}
