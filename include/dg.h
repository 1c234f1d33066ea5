/*
 * dg.h -- C ABI of the discontinuous-Galerkin volume term for the 2D
 * shallow-water equations in libsem.so: the third example of Medina,
 * St-Cyr & Warburton, "OCCA: A unified approach to multi-threading
 * languages" (arXiv 1403.0968), section 4.3 (the volume kernel its
 * section 4.3.3 profiles).
 *
 * Equations (section 4.3.1, equation dgPDE): Q_t + F_x + G_y = S with
 * Q = (h, hu, hv), F = (hu, hu^2/h + g h^2/2, hu hv/h),
 * G = (hv, hu hv/h, hv^2/h + g h^2/2), S = (0, -g h B_x, -g h B_y).
 * Discretisation (section 4.3.2): conforming triangles, Q in P^N per element
 * with a nodal basis; the volume kernel is, for every test function v,
 * <F, v_x> + <G, v_y> + <S, v> on the element.  dg_volume returns it after
 * the inverse mass matrix, as nodal values: with the nodal interpolants of
 * F, G and S,
 *     rhs = Dxw F + Dyw G + S,  Dxw = M^-1 Dx^T M,  Dyw = M^-1 Dy^T M.
 *
 * Reference triangle (-1,-1), (1,-1), (-1,1); warp-and-blend nodes
 * (Warburton 2006, the nodal-DG textbook's construction with its optimised
 * blending parameters), Np = (N+1)(N+2)/2 per element, ordered in rows
 * n = 0..N from the edge s = -1 and m = 0..N-n along each row
 * (dg_reference_nodes).  Elements are affine: x = -(r+s)/2 x1 + (1+r)/2 x2
 * + (1+s)/2 x3 for the element's vertices (x1, x2, x3) in counterclockwise
 * order.  Nodal arrays are [E][Np]; the state and the result are
 * [E][3][Np] (h, hu, hv blocks per element), FP64.
 *
 * Conventions as in sem.h (sem_status errors, sem_last_error, streams).
 */
#ifndef DG_H
#define DG_H
#include <stdint.h>

#include "sem.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_handle dg_handle; /* opaque, owned by the library */

/* Reference nodes (r[Np], s[Np], HOST arrays) of order N in 1..8: the
 * nodal basis points of section 4.3.2 (warp-and-blend construction).
 * SEM_ERR_ARG for another N or a NULL array. */
sem_status dg_reference_nodes(int32_t N, double *r, double *s);

/* Build a handle for the volume term of section 4.3.2 from a triangle mesh: vx, vy (HOST, n_vertices each), etov
 * (HOST int32 [n_elements][3], counterclockwise, indices < n_vertices),
 * bathymetry (HOST [n_elements][Np] nodal values of B, or NULL for a flat
 * bottom) and the gravity g.  Computes the reference operators, the affine
 * factors (rx, sx, ry, sy) and the bathymetry gradient (derivatives of B's
 * nodal interpolant), and uploads them.  SEM_ERR_ARG for N outside 1..8,
 * out-of-range vertex indices, clockwise or degenerate elements, or a
 * non-finite g.  Synchronises `stream`. */
sem_status dg_setup(int32_t N, int64_t n_vertices, const double *vx,
                    const double *vy, int64_t n_elements, const int32_t *etov,
                    const double *bathymetry, double g, void *stream,
                    dg_handle **out);
/* Release a handle of the section 4.3.2 volume term and its device
 * buffers.  NULL is accepted. */
sem_status dg_destroy(dg_handle *h);
/* Nodes per element Np = (N+1)(N+2)/2 and the element count of the
 * section 4.3.2 discretisation (HOST outputs, either may be NULL). */
sem_status dg_query(const dg_handle *h, int32_t *n_nodes, int64_t *n_elements);

/* Copy an internal array of the section 4.3.2 discretisation into caller
 * DEVICE memory, for checking (SEM_ERR_ARG when dst_bytes is too small):
 *   DG_ARR_X, DG_ARR_Y  double [E][Np]   physical node coordinates
 *   DG_ARR_GEO          double [E][4]    (rx, sx, ry, sy)
 *   DG_ARR_DB           double [E][2][Np] (B_x block, B_y block)
 *   DG_ARR_DRW, DG_ARR_DSW double [Np][Np] weak derivative matrices */
typedef enum {
  DG_ARR_X = 0, DG_ARR_Y = 1, DG_ARR_GEO = 2, DG_ARR_DB = 3, DG_ARR_DRW = 4,
  DG_ARR_DSW = 5
} dg_array;
sem_status dg_export(const dg_handle *h, int32_t which, void *dst,
                     int64_t dst_bytes, void *stream);

/* Volume term of section 4.3.2 (the kernel section 4.3.3 profiles),
 * rhs = Dxw F + Dyw G + S, for the state Q (DEVICE, [E][3][Np],
 * h > 0) into rhs (DEVICE, [E][3][Np], must not overlap Q).  FP64 on the
 * matrix cores; asynchronous on `stream`. */
sem_status dg_volume(dg_handle *h, const double *Q, double *rhs, void *stream);

/* The same volume term of section 4.3.2 with the state and the result in
 * blocks of 16 elements, element fastest: component c (0 h, 1 hu, 2 hv) of
 * node n of element e is entry ((e / 16 * 3 + c) * Np + n) * 16 + e % 16.
 * Q and rhs (DEVICE) hold ceil(E / 16) * 16 * 3 * Np doubles each and must
 * not overlap; the entries of the padding elements of the last block
 * (e >= E) are neither read nor written.  Results equal dg_volume's bit
 * for bit; every load and store of the kernel covers whole cache lines.
 * Asynchronous on `stream`. */
sem_status dg_volume_blocked(dg_handle *h, const double *Q, double *rhs,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif
