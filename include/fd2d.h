/*
 * fd2d.h -- C ABI of the finite-difference wave-equation step in libsem.so:
 * the first example of Medina, St-Cyr & Warburton, "OCCA: A unified approach
 * to multi-threading languages" (arXiv 1403.0968), section 4.1 (its
 * pseudocode and kernel fd2d).
 *
 * Problem (section 4.1.1): u_tt = u_xx + u_yy with sound speed 1 on the
 * square [-1, 1]^2.  Discretisation (section 4.1.2): a periodic grid of
 * nx x ny nodes, node (i, j) at index j * nx + i (i fastest), time stepping
 * by the three-point stencil {1, -2, 1} / dt^2 and a central stencil of
 * 2r + 1 nodes (order 2r) per direction in space:
 *
 *   u_next(i,j) = 2 u_cur(i,j) - u_prev(i,j)
 *                 + (dt^2 / dx^2) sum_{k=-r..r} w_k (u_cur(i+k,j) + u_cur(i,j+k))
 *
 * with indices taken modulo nx and ny.  The printed update of the paper
 * carries the opposite sign on every term, which does not define a stable
 * scheme; this is the leapfrog step its stated time stencil defines.
 *
 * Conventions as in sem.h: grid arrays are DEVICE pointers to double owned
 * by the caller, calls are asynchronous on `stream` (a hipStream_t, NULL =
 * the null stream), errors return a sem_status and sem_last_error() gives
 * the text.
 */
#ifndef FD2D_H
#define FD2D_H
#include <stdint.h>

#include "sem.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Unit-spacing weights of the second derivative, order 2r, into the HOST
 * array w[2r + 1] (w[r + k] = w_k, k = -r..r): w_k = 2 (-1)^(k+1) (r!)^2 /
 * (k^2 (r-k)! (r+k)!) for k != 0, w_0 = -2 sum_{k>0} w_k.  r in 1..7
 * (stencil sizes 3..15, the range of section 4.1.3); SEM_ERR_ARG otherwise. */
sem_status fd2d_weights(int32_t r, double *w);

/* One time step of the section 4.1.2 scheme (the paper's kernel fd2d):
 * u_next from u_cur (time level n) and u_prev (level n-1),
 * each nx * ny doubles.  u_next may be the same buffer as u_prev (each node
 * of u_prev is read only to produce the same node of u_next) but must not
 * overlap u_cur.  nx, ny >= 1, r in 1..7, dx > 0, dt and dx finite;
 * SEM_ERR_ARG otherwise. */
sem_status fd2d_step(const double *u_cur, const double *u_prev, double *u_next,
                     int64_t nx, int64_t ny, int32_t r, double dt, double dx,
                     void *stream);

/* nsteps time steps of the section 4.1.2 scheme on two buffers, in place
 * (the paper's driver rotates three buffers, section 4.1.2): on entry u_a holds level n-1
 * and u_b level n; each step overwrites the older level.  On return, after
 * an even number of steps u_a holds level n+nsteps-1 and u_b level n+nsteps;
 * after an odd number the two are swapped (u_a holds the newest).  The same
 * argument rules as fd2d_step; nsteps >= 0. */
sem_status fd2d_run(double *u_a, double *u_b, int64_t nx, int64_t ny, int32_t r,
                    double dt, double dx, int32_t nsteps, void *stream);

#ifdef __cplusplus
}
#endif
#endif
