/*
 * sem_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Every routine is written as the plain definition or as the
 * paper's/textbook's steps in order, with no blocking or fusion, so that it
 * can be checked by eye against:
 *
 *   - the screened-Coulomb problem and its weak form (paper section 4.2 and
 *     4.2.1, equations semPDE and semOperator), with alpha = 0;
 *   - the tensor-product Lagrange basis on 1D Gauss-Lobatto-Legendre nodes
 *     (section 4.2.1) and the diagonal lumped mass J w_abc obtained from
 *     discrete orthogonality (section 4.2.1, first display);
 *   - the derivative sparsity of the tensor basis at the nodes and the chain
 *     rule u_x = r_x u_r + s_x u_s + t_x u_t (section 4.2.1);
 *   - the factored stiffness action with G^T G between reference gradients,
 *     precomputed per elemental node (section 4.2.1, last display);
 *   - distinct global-local numbering / direct stiffness summation
 *     (section 4.2.1, citing Fischer 1991) and PCG (section 4.2.2);
 *   - GLL nodes, weights and the nodal derivative matrix in their standard
 *     closed forms (Deville, Fischer & Mund, cited in section 4.2.1).
 *
 * Compile with -ffp-contract=off: no fused multiply-add, no fast-math.
 */
#include "sem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops that follow (harness control for timing;
 * no result depends on it: every parallel loop writes disjoint outputs). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void orc_legendre(int n, double x, double *P) {
  /* (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} */
  P[0] = 1.0;
  if (n >= 1) P[1] = x;
  for (int k = 1; k < n; ++k)
    P[k + 1] = ((2.0 * k + 1.0) * x * P[k] - k * P[k - 1]) / (k + 1.0);
}

/* GLL nodes: the end points -1, 1 and the N-1 roots of P_N'.  Newton is run
 * on q(x) = (1-x^2) P_N'(x), which equals N (P_{N-1}(x) - x P_N(x)), and whose
 * derivative is -N(N+1) P_N(x) by Legendre's equation.  Start values are the
 * Chebyshev-Gauss-Lobatto points -cos(pi i / N).  Weights are
 * 2 / (N (N+1) P_N(xi)^2). */
int orc_gll(int N, double *xi, double *w) {
  if (N < 1 || N > 32) return -1;
  double P[34];
  int maxit_used = 0;
  xi[0] = -1.0;
  xi[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double x = -cos(ORC_PI * i / N);
    int it;
    for (it = 0; it < 100; ++it) {
      orc_legendre(N, x, P);
      double q = N * (P[N - 1] - x * P[N]);
      double dq = -N * (N + 1.0) * P[N];
      double dx = -q / dq;
      x += dx;
      if (fabs(dx) < 1e-16) break;
    }
    if (it == 100) return -1;
    if (it + 1 > maxit_used) maxit_used = it + 1;
    xi[i] = x;
  }
  /* exact symmetry xi_{N-i} = -xi_i, midpoint exactly 0 */
  for (int i = 0; i <= N / 2; ++i) {
    double s = 0.5 * (xi[N - i] - xi[i]);
    xi[i] = -s;
    xi[N - i] = s;
  }
  if (N % 2 == 0) xi[N / 2] = 0.0;
  for (int i = 0; i <= N; ++i) {
    orc_legendre(N, xi[i], P);
    w[i] = 2.0 / (N * (N + 1.0) * P[N] * P[N]);
  }
  return maxit_used;
}

/* D_ij = l_j'(xi_i): off-diagonal P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)),
 * D_00 = -N(N+1)/4, D_NN = N(N+1)/4, other diagonal entries 0. */
void orc_dmat(int N, const double *xi, double *D) {
  int n1 = N + 1;
  double P[34], PN[34];
  for (int i = 0; i < n1; ++i) {
    orc_legendre(N, xi[i], P);
    PN[i] = P[N];
  }
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      double v;
      if (i != j)
        v = PN[i] / (PN[j] * (xi[i] - xi[j]));
      else if (i == 0)
        v = -N * (N + 1.0) / 4.0;
      else if (i == N)
        v = N * (N + 1.0) / 4.0;
      else
        v = 0.0;
      D[i * n1 + j] = v;
    }
}

/* Periodic directions (bit 1 x, 2 y, 4 z) identify the faces at 0 and 1:
 * the lattice coordinate E_d N wraps to 0, so that direction has E_d N
 * distinct coordinates instead of E_d N + 1 (the global numbering of the
 * distinct nodes, section 4.2.1, on a periodic box). */
static int64_t orc_lattice(int E, int N, int per) { return (int64_t)E * N + (per ? 0 : 1); }

int64_t orc_num_global(int N, int ex, int ey, int ez, int periodic) {
  return orc_lattice(ex, N, periodic & 1) * orc_lattice(ey, N, periodic & 2) *
         orc_lattice(ez, N, periodic & 4);
}

void orc_maps(int N, int ex, int ey, int ez, int dirichlet, int periodic,
              int32_t *l2g, int32_t *perm, int32_t *offsets, int32_t *mult,
              uint8_t *bmask) {
  const int n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  const int64_t Gx = orc_lattice(ex, N, periodic & 1),
                Gy = orc_lattice(ey, N, periodic & 2),
                Gz = orc_lattice(ez, N, periodic & 4);
  const int64_t E = (int64_t)ex * ey * ez;
  const int64_t nL = E * n3, nG = Gx * Gy * Gz;

  for (int64_t e = 0; e < E; ++e) {
    int64_t exi = e % ex, eyi = (e / ex) % ey, ezi = e / ((int64_t)ex * ey);
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          int64_t l = e * n3 + i + (int64_t)n1 * j + (int64_t)n1 * n1 * k;
          /* the coordinate E_d N of a periodic direction is coordinate 0 */
          int64_t gx = (exi * N + i) % Gx, gy = (eyi * N + j) % Gy,
                  gz = (ezi * N + k) % Gz;
          l2g[l] = (int32_t)(gx + Gx * (gy + Gy * gz));
          /* Dirichlet faces: the outer faces of the non-periodic directions */
          int onb = (!(periodic & 1) && (gx == 0 || gx == Gx - 1)) ||
                    (!(periodic & 2) && (gy == 0 || gy == Gy - 1)) ||
                    (!(periodic & 4) && (gz == 0 || gz == Gz - 1));
          bmask[l] = (uint8_t)(dirichlet && onb);
        }
  }
  /* counting sort by g, stable in l: gives the (g, l) order */
  int32_t *cnt = (int32_t *)calloc((size_t)nG + 1, sizeof(int32_t));
  for (int64_t l = 0; l < nL; ++l) cnt[l2g[l] + 1]++;
  offsets[0] = 0;
  for (int64_t g = 0; g < nG; ++g) offsets[g + 1] = offsets[g] + cnt[g + 1];
  for (int64_t g = 0; g < nG; ++g) cnt[g] = offsets[g];
  for (int64_t l = 0; l < nL; ++l) perm[cnt[l2g[l]]++] = (int32_t)l;
  for (int64_t l = 0; l < nL; ++l)
    mult[l] = offsets[l2g[l] + 1] - offsets[l2g[l]];
  free(cnt);
}

void orc_coords(int N, int ex, int ey, int ez, int mapping, const double *xi,
                double *X) {
  const int n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  const int64_t E = (int64_t)ex * ey * ez, nL = E * n3;
  const double hx = 1.0 / ex, hy = 1.0 / ey, hz = 1.0 / ez;
  for (int64_t e = 0; e < E; ++e) {
    int64_t exi = e % ex, eyi = (e / ex) % ey, ezi = e / ((int64_t)ex * ey);
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          int64_t l = e * n3 + i + (int64_t)n1 * j + (int64_t)n1 * n1 * k;
          double x = exi * hx + (xi[i] + 1.0) * 0.5 * hx;
          double y = eyi * hy + (xi[j] + 1.0) * 0.5 * hy;
          double z = ezi * hz + (xi[k] + 1.0) * 0.5 * hz;
          double sx = sin(2.0 * ORC_PI * x), sy = sin(2.0 * ORC_PI * y),
                 sz = sin(2.0 * ORC_PI * z);
          double Xx = x, Xy = y, Xz = z;
          if (mapping == ORC_MAP_SINE_X) {
            Xx = x + 0.05 * sy * sz;
          } else if (mapping == ORC_MAP_SINE_CYCLIC) {
            Xx = x + 0.05 * sy * sz;
            Xy = y + 0.05 * sz * sx;
            Xz = z + 0.05 * sx * sy;
          }
          X[l] = Xx;
          X[nL + l] = Xy;
          X[2 * nL + l] = Xz;
        }
  }
}

/* Isoparametric geometry.  At each node the Jacobian matrix
 * Jm[a][b] = d X_a / d r_b is obtained by applying D along direction b to the
 * nodal coordinates; J = det Jm; the rows of Jm^{-1} are grad r, grad s,
 * grad t; G_ab = w_i w_j w_k J kappa (grad r_a . grad r_b) and the lumped mass
 * is B = w_i w_j w_k J. */
void orc_geom(int N, int64_t E, const double *w, const double *D,
              const double *X, const double *kappa, double *G, double *B,
              double *minJ) {
  const int n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  const int64_t nL = E * n3;
  double mj = 1e300;
  for (int64_t e = 0; e < E; ++e) {
    const int64_t base = e * n3;
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const int64_t p = i + (int64_t)n1 * j + (int64_t)n1 * n1 * k;
          double Jm[3][3];
          for (int a = 0; a < 3; ++a) {
            const double *Xa = X + a * nL + base;
            double dr = 0, ds = 0, dt = 0;
            for (int m = 0; m < n1; ++m) {
              dr += D[i * n1 + m] * Xa[m + n1 * j + n1 * n1 * k];
              ds += D[j * n1 + m] * Xa[i + n1 * m + n1 * n1 * k];
              dt += D[k * n1 + m] * Xa[i + n1 * j + n1 * n1 * m];
            }
            Jm[a][0] = dr;
            Jm[a][1] = ds;
            Jm[a][2] = dt;
          }
          /* determinant and inverse by cofactors */
          double c00 = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
          double c01 = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
          double c02 = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
          double det = Jm[0][0] * c00 + Jm[0][1] * c01 + Jm[0][2] * c02;
          double inv[3][3];
          inv[0][0] = c00 / det;
          inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
          inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
          inv[1][0] = c01 / det;
          inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
          inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
          inv[2][0] = c02 / det;
          inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
          inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
          /* inv[b][a] = d r_b / d x_a, so row b of inv is grad r_b */
          double wq = w[i] * w[j] * w[k];
          double kap = kappa ? kappa[base + p] : 1.0;
          double scale = wq * det * kap;
          const int pairs[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
          for (int q = 0; q < 6; ++q) {
            int a = pairs[q][0], b = pairs[q][1];
            double dot = inv[a][0] * inv[b][0] + inv[a][1] * inv[b][1] +
                         inv[a][2] * inv[b][2];
            G[e * 6 * n3 + q * n3 + p] = scale * dot;
          }
          B[base + p] = wq * det;
          if (det < mj) mj = det;
        }
  }
  if (minJ) *minJ = mj;
}

/* w = D^T G D u per element:
 *   u_r(ijk) = sum_m D_im u(mjk), u_s = sum_m D_jm u(imk), u_t = sum_m D_km u(ijm)
 *   [w_r, w_s, w_t] = G [u_r, u_s, u_t]   (G symmetric 3x3 per node)
 *   w(ijk) = sum_m D_mi w_r(mjk) + sum_m D_mj w_s(imk) + sum_m D_mk w_t(ijm) */
static void ax_element(int n1, const double *D, const double *Ge,
                       const double *ue, double *we, double *wr, double *ws,
                       double *wt, int absval) {
  const int n3 = n1 * n1 * n1;
#define IDX(i, j, k) ((i) + n1 * (j) + n1 * n1 * (k))
#define DV(a, b) (absval ? fabs(D[(a) * n1 + (b)]) : D[(a) * n1 + (b)])
  for (int k = 0; k < n1; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) {
        double ur = 0, us = 0, ut = 0;
        for (int m = 0; m < n1; ++m) {
          double a = ue[IDX(m, j, k)], b = ue[IDX(i, m, k)], c = ue[IDX(i, j, m)];
          if (absval) {
            a = fabs(a);
            b = fabs(b);
            c = fabs(c);
          }
          ur += DV(i, m) * a;
          us += DV(j, m) * b;
          ut += DV(k, m) * c;
        }
        int p = IDX(i, j, k);
        double g[6];
        for (int q = 0; q < 6; ++q) {
          g[q] = Ge[q * n3 + p];
          if (absval) g[q] = fabs(g[q]);
        }
        wr[p] = g[0] * ur + g[1] * us + g[2] * ut;
        ws[p] = g[1] * ur + g[3] * us + g[4] * ut;
        wt[p] = g[2] * ur + g[4] * us + g[5] * ut;
      }
  for (int k = 0; k < n1; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) {
        double s = 0;
        for (int m = 0; m < n1; ++m) {
          s += DV(m, i) * wr[IDX(m, j, k)];
          s += DV(m, j) * ws[IDX(i, m, k)];
          s += DV(m, k) * wt[IDX(i, j, m)];
        }
        we[IDX(i, j, k)] = s;
      }
#undef IDX
#undef DV
}

static void ax_all(int N, int64_t E, const double *D, const double *G,
                   const double *u, double *w, int absval) {
  const int n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
#pragma omp parallel
  {
    double *tmp = (double *)malloc(3 * n3 * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t e = 0; e < E; ++e)
      ax_element(n1, D, G + e * 6 * n3, u + e * n3, w + e * n3, tmp, tmp + n3,
                 tmp + 2 * n3, absval);
    free(tmp);
  }
}

void orc_ax(int N, int64_t E, const double *D, const double *G,
            const double *u, double *w) {
  ax_all(N, E, D, G, u, w, 0);
}

void orc_ax_abs(int N, int64_t E, const double *D, const double *G,
                const double *u, double *w) {
  ax_all(N, E, D, G, u, w, 1);
}

/* Q Q^T: pass 1 sums every local copy into its global node in ascending l;
 * pass 2 copies the sum back to every local copy; then Dirichlet nodes are
 * zeroed. */
void orc_gs(int64_t nL, int64_t nG, const int32_t *l2g, const uint8_t *bmask,
            double *v, double *acc) {
  for (int64_t g = 0; g < nG; ++g) acc[g] = 0.0;
  for (int64_t l = 0; l < nL; ++l) acc[l2g[l]] += v[l];
  for (int64_t l = 0; l < nL; ++l) v[l] = bmask[l] ? 0.0 : acc[l2g[l]];
}

/* Diagonal of each local stiffness matrix:
 *   sum_m D_mi^2 G_rr(mjk) + sum_m D_mj^2 G_ss(imk) + sum_m D_mk^2 G_tt(ijm)
 *   + 2 D_ii D_jj G_rs(ijk) + 2 D_ii D_kk G_rt(ijk) + 2 D_jj D_kk G_st(ijk). */
void orc_diag(int N, int64_t E, const double *D, const double *G,
              double *diag) {
  const int n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  for (int64_t e = 0; e < E; ++e) {
    const double *Ge = G + e * 6 * n3;
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          double s = 0;
          for (int m = 0; m < n1; ++m) {
            double dmi = D[m * n1 + i], dmj = D[m * n1 + j], dmk = D[m * n1 + k];
            s += dmi * dmi * Ge[0 * n3 + m + n1 * j + n1 * n1 * k];
            s += dmj * dmj * Ge[3 * n3 + i + n1 * m + n1 * n1 * k];
            s += dmk * dmk * Ge[5 * n3 + i + n1 * j + n1 * n1 * m];
          }
          int p = i + n1 * j + n1 * n1 * k;
          double di = D[i * n1 + i], dj = D[j * n1 + j], dk = D[k * n1 + k];
          s += 2.0 * di * dj * Ge[1 * n3 + p];
          s += 2.0 * di * dk * Ge[2 * n3 + p];
          s += 2.0 * dj * dk * Ge[4 * n3 + p];
          diag[e * n3 + p] = s;
        }
  }
}

void orc_src_fourier(int64_t n, const double *X, int nm, const double *k,
                     const double *a, const double *phi, double *f) {
  for (int64_t l = 0; l < n; ++l) {
    double x = X[l], y = X[n + l], z = X[2 * n + l];
    double s = 0;
    for (int m = 0; m < nm; ++m)
      s += a[m] * cos(2.0 * ORC_PI * (k[3 * m] * x + k[3 * m + 1] * y +
                                       k[3 * m + 2] * z) + phi[m]);
    f[l] = s;
  }
}

void orc_src_sine(int64_t n, const double *X, double *f) {
  for (int64_t l = 0; l < n; ++l)
    f[l] = 3.0 * ORC_PI * ORC_PI * sin(ORC_PI * X[l]) * sin(ORC_PI * X[n + l]) *
           sin(ORC_PI * X[2 * n + l]);
}

void orc_kappa_rff(int64_t n, const double *X, int M, const double *omega,
                   const double *b, double sigma, double *kappa) {
  const double c = sigma * sqrt(2.0 / M);
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < n; ++l) {
    double x = X[l], y = X[n + l], z = X[2 * n + l];
    double s = 0;
    for (int m = 0; m < M; ++m)
      s += cos(omega[3 * m] * x + omega[3 * m + 1] * y + omega[3 * m + 2] * z +
               b[m]);
    kappa[l] = exp(c * s);
  }
}

void orc_apply_global(int N, int64_t E, int64_t nG, const int32_t *l2g,
                      const uint8_t *bmask, const double *D, const double *G,
                      const double *H, const double *x, double *y) {
  const int64_t n1 = N + 1, nL = E * n1 * n1 * n1;
  double *xl = (double *)calloc((size_t)nL, sizeof(double));
  double *yl = (double *)malloc(nL * sizeof(double));
  for (int64_t l = 0; l < nL; ++l) xl[l] = bmask[l] ? 0.0 : x[l2g[l]];
  orc_ax(N, E, D, G, xl, yl);
  /* lumped mass term of the weak form: alpha(X) w J at each local node */
  if (H)
    for (int64_t l = 0; l < nL; ++l) yl[l] += H[l] * xl[l];
  for (int64_t g = 0; g < nG; ++g) y[g] = 0.0;
  for (int64_t l = 0; l < nL; ++l) y[l2g[l]] += yl[l];
  for (int64_t l = 0; l < nL; ++l)
    if (bmask[l]) y[l2g[l]] = 0.0;
  free(xl);
  free(yl);
}

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Textbook preconditioned conjugate gradients (Hestenes-Stiefel; Saad,
 * Iterative Methods, Algorithm 9.1) with x0 taken from x. */
int orc_pcg(int N, int64_t E, int64_t nG, const int32_t *l2g,
            const uint8_t *bmask, const double *D, const double *G,
            const double *H, const double *dinv, const double *b, double *x,
            double rtol, int maxit, int *iters, double *hist) {
  double *r = (double *)malloc(nG * sizeof(double));
  double *z = (double *)malloc(nG * sizeof(double));
  double *p = (double *)malloc(nG * sizeof(double));
  double *w = (double *)malloc(nG * sizeof(double));
  int status = 1, k = 0;
  orc_apply_global(N, E, nG, l2g, bmask, D, G, H, x, w);
  for (int64_t g = 0; g < nG; ++g) r[g] = b[g] - w[g];
  const double bnorm = sqrt(dot(nG, b, b));
  double rnorm = sqrt(dot(nG, r, r));
  if (hist) hist[0] = bnorm > 0 ? rnorm / bnorm : 0.0;
  if (rnorm <= rtol * bnorm) {
    status = 0;
    goto done;
  }
  for (int64_t g = 0; g < nG; ++g) z[g] = dinv ? dinv[g] * r[g] : r[g];
  for (int64_t g = 0; g < nG; ++g) p[g] = z[g];
  double rz = dot(nG, r, z);
  for (k = 1; k <= maxit; ++k) {
    orc_apply_global(N, E, nG, l2g, bmask, D, G, H, p, w);
    double pw = dot(nG, p, w);
    if (!(pw > 0)) {
      status = 2;
      break;
    }
    double alpha = rz / pw;
    for (int64_t g = 0; g < nG; ++g) x[g] += alpha * p[g];
    for (int64_t g = 0; g < nG; ++g) r[g] -= alpha * w[g];
    rnorm = sqrt(dot(nG, r, r));
    if (hist) hist[k] = rnorm / bnorm;
    if (rnorm <= rtol * bnorm) {
      status = 0;
      break;
    }
    for (int64_t g = 0; g < nG; ++g) z[g] = dinv ? dinv[g] * r[g] : r[g];
    double rz_new = dot(nG, r, z);
    double beta = rz_new / rz;
    rz = rz_new;
    for (int64_t g = 0; g < nG; ++g) p[g] = z[g] + beta * p[g];
  }
  if (k > maxit) k = maxit;
done:
  if (iters) *iters = k;
  free(r);
  free(z);
  free(p);
  free(w);
  return status;
}

/* Flexible CG for a preconditioner that may change between iterations
 * (Notay 2000, truncated to one previous direction): the new direction is
 * z_{k+1} A-orthogonalised against p_k,
 *   p_{k+1} = z_{k+1} + beta p_k,  beta = -(z_{k+1}, A p_k) / (p_k, A p_k),
 * and alpha = (r_k, z_k) / (p_k, A p_k). */
int orc_fcg(int N, int64_t E, int64_t nG, const int32_t *l2g,
            const uint8_t *bmask, const double *D, const double *G,
            const double *H, orc_precond_fn prec, void *ctx, const double *b,
            double *x, double rtol, int maxit, int *iters, double *hist) {
  double *r = (double *)malloc(nG * sizeof(double));
  double *z = (double *)malloc(nG * sizeof(double));
  double *p = (double *)malloc(nG * sizeof(double));
  double *w = (double *)malloc(nG * sizeof(double));
  int status = 1, k = 0;
  orc_apply_global(N, E, nG, l2g, bmask, D, G, H, x, w);
  for (int64_t g = 0; g < nG; ++g) r[g] = b[g] - w[g];
  const double bnorm = sqrt(dot(nG, b, b));
  double rnorm = sqrt(dot(nG, r, r));
  if (hist) hist[0] = bnorm > 0 ? rnorm / bnorm : 0.0;
  if (rnorm <= rtol * bnorm) {
    status = 0;
    goto done;
  }
  prec(r, z, ctx);
  for (int64_t g = 0; g < nG; ++g) p[g] = z[g];
  for (k = 1; k <= maxit; ++k) {
    orc_apply_global(N, E, nG, l2g, bmask, D, G, H, p, w);
    double pw = dot(nG, p, w);
    double rz = dot(nG, r, z);
    if (!(pw > 0)) {
      status = 2;
      break;
    }
    double alpha = rz / pw;
    for (int64_t g = 0; g < nG; ++g) x[g] += alpha * p[g];
    for (int64_t g = 0; g < nG; ++g) r[g] -= alpha * w[g];
    rnorm = sqrt(dot(nG, r, r));
    if (hist) hist[k] = rnorm / bnorm;
    if (rnorm <= rtol * bnorm) {
      status = 0;
      break;
    }
    prec(r, z, ctx);
    double beta = -dot(nG, z, w) / pw;
    for (int64_t g = 0; g < nG; ++g) p[g] = z[g] + beta * p[g];
  }
  if (k > maxit) k = maxit;
done:
  if (iters) *iters = k;
  free(r);
  free(z);
  free(p);
  free(w);
  return status;
}
