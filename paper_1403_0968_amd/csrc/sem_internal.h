// Internal declarations of libsem.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "../../include/sem.h"
#include "structured.h"

namespace sem {

// ---------------------------------------------------------------------------
// error plumbing: internal code throws sem::Error, the C ABI converts it
// ---------------------------------------------------------------------------
struct Error {
  sem_status code;
  std::string msg;
};
[[noreturn]] void fail(sem_status code, const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define SEM_HIP(x) ::sem::hip_check((x), #x, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// reference element (host, FP64)
// ---------------------------------------------------------------------------
struct RefElem {
  int N = 0, n1 = 0;
  std::vector<double> xi, w, D;  // D[i*n1+m] = l_m'(xi_i)
};
RefElem make_ref_elem(int N);

// reference triangle of the DG volume term (host, FP64, row-major Np x Np)
struct DgRef {
  int N = 0, Np = 0;
  std::vector<double> r, s, Dr, Ds, Drw, Dsw;
};
DgRef make_dg_ref(int N);

// ---------------------------------------------------------------------------
// maps of the structured box (host)
// ---------------------------------------------------------------------------
struct HostMaps {
  int64_t nL = 0, nG = 0;
  std::vector<int32_t> l2g, perm, offsets, mult;
  std::vector<uint8_t> bmask;   // per local node, 1 on Dirichlet nodes
  std::vector<uint8_t> gmask;   // per global node
};
// periodic: bit 1 x, 2 y, 4 z (faces at 0 and 1 identified)
HostMaps make_maps(int N, int ex, int ey, int ez, int dirichlet, int periodic);

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  bool own = true;  // false: a view of memory owned elsewhere (never freed)
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf();
  void alloc(size_t nbytes);
  void view(void *q, size_t nbytes);
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// device-side CG scalars (one struct per solve)
struct CgState {
  double rz;      // (r, z)
  double pw;      // (p, A p)
  double alpha, beta;
  double rr;      // (r, r)
  double bb;      // (b, b)
  double tol2;    // rtol^2
  double pad0;
  int32_t it;     // iterations done
  int32_t maxit;
  int32_t done;   // 0 running, 1 converged, 2 breakdown, 3 maxit, 4 idle
  int32_t xupd;   // 1: this iteration's x += alpha p is still to be applied
};

// vectors of one solve (unique-node layout except VWL, an E-vector)
enum { VB = 0, VX, VR, VZ, VP, VW, VWL, NVEC };

// one solve of a batch as the device kernels see it
struct BatchSolve {
  int32_t N1, solve;
  int64_t E, nL, nG;
  Box box;                        // closed-form numbering of the solve's mesh
  const void *G64, *G32, *G16, *D64, *D32;
  const void *D16hi, *D16lo;      // two-term BF16 split of D
  const void *H16;                // BF16 mass factor alpha B, or null
  const double *dinv64, *one64;   // Jacobi, and 1 off the Dirichlet boundary
  const float *dinv32, *one32;
  void *v64[NVEC];
  void *v32[NVEC];
  double *edot;                   // [E] element energies p_e^T (A p)_e
};

// work items of the persistent kernels
struct AxItem {  // a tile of elements of one solve
  int32_t solve, pad;
  int64_t elem0;
};
struct VecItem {  // a chunk of unique nodes of one solve
  int32_t solve, pad;
  int64_t start;
};
// unique nodes per vector item (one workgroup of a vector kernel, four per
// thread; against 2048 at 32^3 and 24^3, N = 7: FP64 iteration 345.4 ->
// 342.3 and 164.7 -> 161.3 us, 4^3 mesh 30.8 -> 28.5 us, the loop of 256
// small solves 10.9 -> 10.3 s; 512 and 4096 were slower)
constexpr int VCH = 1024;
constexpr int AX_SET_468 = 100;  // batched operator compiled for n1 in {4,6,8}

}  // namespace sem

struct dg_handle {
  int N = 0, Np = 0;
  int64_t E = 0;
  double g = 0.0;
  sem::DgRef ref;
  // per element: (rx, sx, ry, sy); bathymetry gradient [E][2][Np] and in
  // blocks of 16 elements [E/16][2][Np][16]; node coordinates [E][Np]; Drw,
  // Dsw zero-padded to whole MFMA tiles and stored in the lane order of the
  // volume kernel's matrix instruction
  sem::DevBuf geo, dB, dBb, X, Y, Drw, Dsw;
};

namespace sem {
struct Workspace;  // solver buffers, graphs and streams (solver.hip)
struct Learn;      // learned-correction buffers (learn.hip)
}

struct sem_handle {
  int N = 0, n1 = 0, ex = 0, ey = 0, ez = 0, dirichlet = 0, mapping = 0;
  int periodic = 0;  // bit 1 x, 2 y, 4 z
  int64_t E = 0, nL = 0, nG = 0;
  sem::RefElem ref;

  // maps
  sem::DevBuf l2g, perm, offsets, mult, bmask, gmask;
  // reference element on device
  sem::DevBuf D64, D32, D16hi, D16lo;  // D16hi + D16lo: BF16 split of D
  // geometry and preconditioner
  sem::DevBuf coords, G64, G32, G16, mass, diag_L, dinv_G, dinv_G32;
  sem::DevBuf kvert;            // kappa at the 8 vertices of each element
  // mass term H = alpha(X) B (allocated only when alpha != 0), FP64 with
  // FP32 / BF16 copies in the natural [E][n1^3] layout
  bool has_mass = false;
  sem::DevBuf H64, H32, H16;
  // created on the first solve
  sem::Workspace *ws = nullptr;
  // learned correction (attached network, element features and scratch)
  sem_mlp *net = nullptr;
  sem::Learn *learn = nullptr;
};

namespace sem {

// kernels / launchers (ax.hip, gs.hip, setup.hip)
// H: mass factor in the precision of G, or null (no mass term)
void launch_ax(int N, int prec, int64_t E, const void *D, const void *G,
               const void *H, const void *u, void *w, hipStream_t s);
void launch_gs(sem_handle *h, int prec, void *v, hipStream_t s);
void device_setup(sem_handle *h, const sem_mesh_desc *d, hipStream_t s);
void launch_rhs(sem_handle *h, const sem_source *src, double *b, hipStream_t s);
void launch_precond(sem_handle *h, int pc, int prec, const void *r, void *z,
                    hipStream_t s);
// persistent batched operator over (solve, element tile) items; src / dst are
// vector indices (VP, VX, ..., VWL) of the precision's vector set
void launch_bax(int prec, int bs, int nset, const BatchSolve *sds,
                const CgState *st, const AxItem *items, int nitems, int grid,
                int src, int dst, int skip_done, hipStream_t s);
// nt: store the output with the streaming hint (vectors beyond the caches)
void launch_ax_solve(int N, int prec, int64_t E, const void *D, const void *G,
                     const void *H, const void *u, void *w, const Box &box,
                     const int32_t *stop, double *edot, bool nt, hipStream_t s);
void launch_ax_mfma(int N, bool split, int64_t E, const uint16_t *Dhi,
                    const uint16_t *Dlo, const uint16_t *G, const uint16_t *H,
                    const uint16_t *u, float *w, hipStream_t s);
void launch_bax_mfma(int n1, bool split, const BatchSolve *sds, const CgState *st,
                     const AxItem *items, int nitems, int epb, int grid, int src,
                     int dst, int skip_done, bool edot, hipStream_t s);
// the matrix-core solver operator of a single solve (gathered FP32 input,
// FP32 output; element energies into edot when non-null)
void launch_ax_mfma_solve(int N, bool split, int64_t E, const uint16_t *Dhi,
                          const uint16_t *Dlo, const uint16_t *G, const uint16_t *H,
                          const float *u, float *w, const Box &box, const int32_t *stop,
                          double *edot, hipStream_t s);
int bax_elements_per_tile(int bs, int n1);
// smallest workgroup (64, 128, 256) holding every (i, j) column of the
// largest order of an order set
int bax_min_block(int nset);
// DG volume term (dg.hip)
void dg_device_setup(dg_handle *h, int64_t nv, const double *vx, const double *vy,
                     const int32_t *etov, const double *B, hipStream_t s);
// blocked: state and result in blocks of 16 elements, [E/16][3][Np][16]
void launch_dg_volume(const dg_handle *h, const double *Q, double *rhs,
                      bool blocked, hipStream_t s);
// finite-difference wave step (fd2d.hip); c = dt^2 / dx^2
void fd2d_weights_host(int r, double *w);
void launch_fd2d(const double *u_cur, const double *u_prev, double *u_next,
                 int64_t nx, int64_t ny, int r, double c, hipStream_t s);
// solver (solver.hip)
void destroy_ws(sem_handle *h);
sem_batch *batch_create(sem_handle *const *hs, int n);
void batch_destroy(sem_batch *b);
void batch_tune(sem_batch *b, int prec, int *best_bs, int *best_gm,
                double *best_us);
sem_status batch_solve(sem_batch *b, const sem_solve_opts *o,
                       const double *const *bL, double *const *xL,
                       sem_solve_stats *stats, hipStream_t caller);
// network (mlp.hip)
sem_mlp *mlp_create(int n_in, int H, int n_out, uint64_t seed);
void mlp_destroy(sem_mlp *net);
void mlp_set_params(sem_mlp *net, const float *host, int64_t n);
void mlp_get_params(const sem_mlp *net, float *host, int64_t n);
void mlp_info(const sem_mlp *net, int *n_in, int *H, int *n_out, int64_t *np,
              int64_t *step);
int mlp_padded_inputs(const sem_mlp *net);
void mlp_refresh(sem_mlp *net, hipStream_t s);
void mlp_forward(sem_mlp *net, const uint16_t *X, int ldx, int B, float *O,
                 int ldo, hipStream_t s);
void mlp_set_precision(sem_mlp *net, int prec);
int mlp_precision(const sem_mlp *net);
double mlp_loss_grad_factor(sem_mlp *net, const uint16_t *X, int ldx,
                            const float *T, int K, int B, bool host_loss,
                            hipStream_t s);
uint64_t mlp_version(const sem_mlp *net);
void mlp_adam(sem_mlp *net, const float *grad, double lr, double b1, double b2,
              double eps, hipStream_t s);
void mlp_save(const sem_mlp *net, const char *path);
sem_mlp *mlp_load(const char *path);
const float *mlp_grad_ptr(const sem_mlp *net);
double mlp_damping(const sem_mlp *net);
double mlp_ref_rate(const sem_mlp *net);
void mlp_set_damping(sem_mlp *net, double damping, double ref_rate);
const float *mlp_damping_dev(const sem_mlp *net);
// learned correction on a mesh (learn.hip)
void learn_attach(sem_handle *h, sem_mlp *net);
void learn_destroy(sem_handle *h);
// one application c = damping B M_e B^T r_I for the batch's single solve
// (r a unique-node vector, FP32 when f32), into the unique-node correction
void learn_apply(sem_handle *h, const void *r, bool f32, hipStream_t s);
void learn_apply_fused(sem_handle *h, const void *r, void *z, const void *wL,
                       bool f32, hipStream_t s);
double *learn_epart(sem_handle *h);
void learn_attach_exact(sem_handle *h, double damping);
bool learn_active(const sem_handle *h);
double learn_damping(const sem_handle *h);
double learn_ref_rate(const sem_handle *h);
void learn_refresh(sem_handle *h);
int learn_coarse_exact(sem_handle *h, double *M, hipStream_t s);
void learn_train(sem_handle *h, sem_mlp *net, const double *const *bL, int nrhs,
                 const sem_train_opts *o, sem_train_report *rep,
                 hipStream_t caller);
sem_status pcg_solve(sem_handle *h, const sem_solve_opts *o, const double *b_L,
                     double *x_L, sem_solve_stats *st, hipStream_t s);
// plain FP64 PCG with every device buffer in a fixed per-GPU array (no
// allocation); noalloc_bytes: the part of the array a handle's solve needs
sem_status pcg_solve_noalloc(sem_handle *h, const sem_solve_opts *o,
                             const double *b_L, double *x_L, sem_solve_stats *st,
                             hipStream_t caller);
size_t noalloc_bytes(const sem_handle *h);

}  // namespace sem
