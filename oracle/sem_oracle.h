/*
 * sem_oracle.h -- plain FP64 CPU oracle for the spectral-element Poisson
 * operator of Medina, St-Cyr & Warburton (arXiv 1403.0968), section 4.2.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the HIP product path is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the product library.
 *
 * Conventions (written down independently by both sides, never shared code):
 *   n1 = N+1 GLL points per direction, element-local node (i,j,k) with i
 *   fastest; element e = ex + Ex*(ey + Ey*ez); local index
 *   l = e*n1^3 + i + n1*j + n1^2*k;  global index
 *   g = (ex*N+i) + Gx*((ey*N+j) + Gy*(ez*N+k)),  Gd = Ed*N+1.
 *   Geometric factors are stored [E][6][n1^3] in the order
 *   (rr, rs, rt, ss, st, tt).
 *
 * Parity status: every function below is pinned by closed forms,
 * invariants or brute force in tests/ (tests/test_oracle_*.py).
 */
#ifndef SEM_ORACLE_H
#define SEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Mappings of the unit cube (affine box, one sine term, cyclic sine terms). */
enum { ORC_MAP_AFFINE = 0, ORC_MAP_SINE_X = 1, ORC_MAP_SINE_CYCLIC = 2 };

/* OpenMP threads the parallel loops use. */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Legendre P_0..P_n at x by the three-term recurrence; P has n+1 entries. */
void orc_legendre(int n, double x, double *P);

/* GLL nodes xi[0..N] and weights w[0..N].  Returns Newton iterations used
 * (max over nodes) or -1 on failure. */
int orc_gll(int N, double *xi, double *w);

/* Nodal derivative matrix D[i*(N+1)+j] = l_j'(xi_i). */
void orc_dmat(int N, const double *xi, double *D);

/* Number of distinct global nodes; periodic: bit 1 x, 2 y, 4 z. */
int64_t orc_num_global(int N, int ex, int ey, int ez, int periodic);

/* Maps: l2g[nL], perm[nL] (local ids sorted by (g,l)), offsets[nG+1],
 * mult[nL] (copies of l's global node), bmask[nL] (1 on Dirichlet nodes,
 * i.e. global nodes on the outer faces of the non-periodic directions when
 * dirichlet != 0).  A periodic direction identifies its faces at 0 and 1. */
void orc_maps(int N, int ex, int ey, int ez, int dirichlet, int periodic,
              int32_t *l2g, int32_t *perm, int32_t *offsets, int32_t *mult,
              uint8_t *bmask);

/* Physical coordinates X[3*nL] (x block, y block, z block) of every local
 * GLL node of the unit cube [0,1]^3 under the chosen mapping. */
void orc_coords(int N, int ex, int ey, int ez, int mapping, const double *xi,
                double *X);

/* Geometric factors G[E][6][n1^3] and lumped mass B[nL] from the nodal
 * coordinates (isoparametric).  kappa may be NULL (kappa = 1).  Returns the
 * minimum Jacobian determinant in *minJ. */
void orc_geom(int N, int64_t E, const double *w, const double *D,
              const double *X, const double *kappa, double *G, double *B,
              double *minJ);

/* Unassembled local stiffness action w = D^T G D u, element by element
 * (OpenMP over elements). */
void orc_ax(int N, int64_t E, const double *D, const double *G,
            const double *u, double *w);
/* Same with |D|, |G|, |u|: the componentwise bound (|A||u|)_l. */
void orc_ax_abs(int N, int64_t E, const double *D, const double *G,
                const double *u, double *w);

/* Direct-stiffness summation Q Q^T v in place (ascending-l order) followed
 * by zeroing of Dirichlet nodes; acc is caller scratch of nG doubles. */
void orc_gs(int64_t nL, int64_t nG, const int32_t *l2g, const uint8_t *bmask,
            double *v, double *acc);

/* Unassembled diagonal of the local stiffness matrices, diag[nL]. */
void orc_diag(int N, int64_t E, const double *D, const double *G,
              double *diag);

/* f(X) = sum_m a_m cos(2 pi k_m . X + phi_m); k is [nm][3]. */
void orc_src_fourier(int64_t n, const double *X, int nm, const double *k,
                     const double *a, const double *phi, double *f);
/* f(X) = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) (manufactured solution). */
void orc_src_sine(int64_t n, const double *X, double *f);
/* kappa(X) = exp(sigma*sqrt(2/M) sum_m cos(omega_m . X + b_m)); omega [M][3]. */
void orc_kappa_rff(int64_t n, const double *X, int M, const double *omega,
                   const double *b, double sigma, double *kappa);

/* Unique-vector operator y = M Q^T A_L Q M x (x, y of length nG).  H, if
 * not NULL, is the lumped mass term alpha(X) B per local node, added to the
 * local operator (A_L = D^T G D + diag(H)). */
void orc_apply_global(int N, int64_t E, int64_t nG, const int32_t *l2g,
                      const uint8_t *bmask, const double *D, const double *G,
                      const double *H, const double *x, double *y);

/* Preconditioned CG on unique vectors (Jacobi when dinv != NULL).  hist, if
 * not NULL, receives ||r_k||/||b|| for k = 0..iters.  Returns 0 on
 * convergence, 1 when maxit is reached, 2 on breakdown. */
int orc_pcg(int N, int64_t E, int64_t nG, const int32_t *l2g,
            const uint8_t *bmask, const double *D, const double *G,
            const double *H, const double *dinv, const double *b, double *x,
            double rtol, int maxit, int *iters, double *hist);

/* Flexible CG with an arbitrary preconditioner callback z = P(r). */
typedef void (*orc_precond_fn)(const double *r, double *z, void *ctx);
int orc_fcg(int N, int64_t E, int64_t nG, const int32_t *l2g,
            const uint8_t *bmask, const double *D, const double *G,
            const double *H, orc_precond_fn prec, void *ctx, const double *b,
            double *x, double rtol, int maxit, int *iters, double *hist);

#ifdef __cplusplus
}
#endif
#endif
