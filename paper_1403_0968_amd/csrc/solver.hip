// Preconditioned conjugate gradients for the assembled SEM system (paper
// section 4.2.2: the system is solved by PCG, whose dominant cost is the
// operator application), plus FP64 iterative refinement around an FP32 /
// BF16-operator inner PCG.
//
// Vectors live on unique (global) nodes; the operator is applied as
//   w_G = mask o Q^T A_L Q p_G
// with Q fused into the operator kernel (gather through l2g) and Q^T + mask
// fused with the (p, w) dot product.  Iteration kernels:
//   ax(gather) -> assemble+dot -> alpha -> x,r update + z = dinv r + dots
//   -> beta/convergence -> p update.
// Scalars stay on the device; each kernel returns at once when the device
// flag says the solve has finished, so a captured graph of K iterations can
// be replayed between host polls without changing the result.  Reductions
// use a fixed grid and a fixed order: results are bit-reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "sem_internal.h"

namespace sem {

constexpr int RT = 256;
constexpr int RBLK_MAX = 2048;

static int red_blocks(int64_t n) {
  int64_t b = (n + RT - 1) / RT;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), RBLK_MAX);
}

// --------------------------------------------------------------------------
// kernels
// --------------------------------------------------------------------------
template <class TL, class TV, bool DOT>
__global__ void __launch_bounds__(RT)
    k_assemble(int64_t nG, const int32_t *__restrict__ off,
               const int32_t *__restrict__ perm,
               const uint8_t *__restrict__ gmask, const TL *__restrict__ wL,
               TV *__restrict__ wG, const TV *__restrict__ p,
               double *__restrict__ part, const int32_t *__restrict__ stop) {
  __shared__ double sm[RT / 64];
  if (stop != nullptr && *stop != 0) return;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RT;
  for (int64_t g = (int64_t)blockIdx.x * RT + threadIdx.x; g < nG; g += stride) {
    TL s = TL(0);
    const int a = off[g], b = off[g + 1];
    for (int q = a; q < b; ++q) s = s + wL[perm[q]];
    const TV v = gmask[g] ? TV(0) : (TV)s;
    wG[g] = v;
    if (DOT) acc += (double)p[g] * (double)v;
  }
  if (DOT) {
    const double t = block_sum<RT>(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(RT)
    k_alpha(CgState *st, const double *__restrict__ part, int nb) {
  __shared__ double sm[RT / 64];
  if (st->done != 0) return;
  double a = 0.0;
  for (int q = threadIdx.x; q < nb; q += RT) a += part[q];
  const double pw = block_sum<RT>(a, sm);
  if (threadIdx.x == 0) {
    st->pw = pw;
    if (!(pw > 0.0) || !isfinite(pw))
      st->done = 2;
    else
      st->alpha = st->rz / pw;
  }
}

template <class TV, class TD>
__global__ void __launch_bounds__(RT)
    k_update_xr(int64_t nG, const CgState *__restrict__ st, TV *__restrict__ x,
                TV *__restrict__ r, const TV *__restrict__ p,
                const TV *__restrict__ w, const TD *__restrict__ dinv,
                TV *__restrict__ z, double *__restrict__ part, int nb) {
  __shared__ double sm[RT / 64];
  if (st->done != 0) return;
  const TV alpha = (TV)st->alpha;
  double rz = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RT;
  for (int64_t g = (int64_t)blockIdx.x * RT + threadIdx.x; g < nG; g += stride) {
    x[g] = x[g] + alpha * p[g];
    const TV rn = r[g] - alpha * w[g];
    r[g] = rn;
    const TV zn = (TV)(dinv[g] * rn);
    z[g] = zn;
    rz += (double)rn * (double)zn;
    rr += (double)rn * (double)rn;
  }
  const double trz = block_sum<RT>(rz, sm);
  const double trr = block_sum<RT>(rr, sm);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = trz;
    part[nb + blockIdx.x] = trr;
  }
}

__global__ void __launch_bounds__(RT)
    k_beta(CgState *st, const double *__restrict__ part, int nb) {
  __shared__ double sm[RT / 64];
  if (st->done != 0) return;
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nb; q += RT) {
    a += part[q];
    b += part[nb + q];
  }
  const double rz = block_sum<RT>(a, sm);
  const double rr = block_sum<RT>(b, sm);
  if (threadIdx.x == 0) {
    st->it += 1;
    st->rr = rr;
    if (!isfinite(rr) || !isfinite(rz))
      st->done = 2;
    else if (rr <= st->tol2 * st->bb)
      st->done = 1;
    else if (st->it >= st->maxit)
      st->done = 3;
    else {
      st->beta = rz / st->rz;
      st->rz = rz;
    }
  }
}

template <class TV>
__global__ void __launch_bounds__(RT)
    k_update_p(int64_t nG, const CgState *__restrict__ st,
               const TV *__restrict__ z, TV *__restrict__ p) {
  if (st->done != 0) return;
  const TV beta = (TV)st->beta;
  const int64_t stride = (int64_t)gridDim.x * RT;
  for (int64_t g = (int64_t)blockIdx.x * RT + threadIdx.x; g < nG; g += stride)
    p[g] = z[g] + beta * p[g];
}

// r = b - w (w == nullptr: x0 = 0, r = b and x is zeroed), z = dinv r, p = z
template <class TV, class TD>
__global__ void __launch_bounds__(RT)
    k_init(int64_t nG, const TV *__restrict__ b, const TV *__restrict__ w,
           TV *__restrict__ x, TV *__restrict__ r, TV *__restrict__ z,
           TV *__restrict__ p, const TD *__restrict__ dinv,
           double *__restrict__ part, int nb) {
  __shared__ double sm[RT / 64];
  double rz = 0.0, rr = 0.0, bb = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RT;
  for (int64_t g = (int64_t)blockIdx.x * RT + threadIdx.x; g < nG; g += stride) {
    const TV bv = b[g];
    TV rv = bv;
    if (w != nullptr)
      rv = bv - w[g];
    else
      x[g] = TV(0);
    const TV zv = (TV)(dinv[g] * rv);
    r[g] = rv;
    z[g] = zv;
    p[g] = zv;
    rz += (double)rv * (double)zv;
    rr += (double)rv * (double)rv;
    bb += (double)bv * (double)bv;
  }
  const double a = block_sum<RT>(rz, sm);
  const double c = block_sum<RT>(rr, sm);
  const double d = block_sum<RT>(bb, sm);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[nb + blockIdx.x] = c;
    part[2 * nb + blockIdx.x] = d;
  }
}

__global__ void __launch_bounds__(RT)
    k_init_reduce(CgState *st, const double *__restrict__ part, int nb,
                  double tol2, int maxit) {
  __shared__ double sm[RT / 64];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int q = threadIdx.x; q < nb; q += RT) {
    a += part[q];
    b += part[nb + q];
    c += part[2 * nb + q];
  }
  const double rz = block_sum<RT>(a, sm);
  const double rr = block_sum<RT>(b, sm);
  const double bb = block_sum<RT>(c, sm);
  if (threadIdx.x == 0) {
    st->rz = rz;
    st->rr = rr;
    st->bb = bb;
    st->tol2 = tol2;
    st->it = 0;
    st->maxit = maxit;
    st->alpha = st->beta = st->pw = 0.0;
    if (!isfinite(rr) || !isfinite(rz))
      st->done = 2;
    else if (rr <= tol2 * bb)
      st->done = 1;
    else if (maxit <= 0)
      st->done = 3;
    else
      st->done = 0;
  }
}

// rr partials of r = b - w (FP64); r is stored when r_out != nullptr
__global__ void __launch_bounds__(RT)
    k_residual(int64_t nG, const double *__restrict__ b,
               const double *__restrict__ w, double *__restrict__ r_out,
               double *__restrict__ part) {
  __shared__ double sm[RT / 64];
  double rr = 0.0, bb = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RT;
  for (int64_t g = (int64_t)blockIdx.x * RT + threadIdx.x; g < nG; g += stride) {
    const double rv = b[g] - w[g];
    if (r_out != nullptr) r_out[g] = rv;
    rr += rv * rv;
    bb += b[g] * b[g];
  }
  const double a = block_sum<RT>(rr, sm);
  const double c = block_sum<RT>(bb, sm);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = c;
  }
}

// out[0] = sum part[0..nb), out[1] = sum part[nb..2nb)
__global__ void __launch_bounds__(RT)
    k_reduce2(const double *__restrict__ part, int nb, double *out) {
  __shared__ double sm[RT / 64];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nb; q += RT) {
    a += part[q];
    b += part[nb + q];
  }
  const double s0 = block_sum<RT>(a, sm);
  const double s1 = block_sum<RT>(b, sm);
  if (threadIdx.x == 0) {
    out[0] = s0;
    out[1] = s1;
  }
}

__global__ void k_scale_cast(int64_t n, const double *__restrict__ r, double s,
                             float *__restrict__ o) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) o[g] = (float)(r[g] * s);
}

__global__ void k_axpy_mixed(int64_t n, double *__restrict__ x,
                             const float *__restrict__ d, double s) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) x[g] += s * (double)d[g];
}

__global__ void k_first_copy(int64_t nG, const int32_t *__restrict__ off,
                             const int32_t *__restrict__ perm,
                             const double *__restrict__ vL,
                             double *__restrict__ vG) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nG) vG[g] = vL[perm[off[g]]];
}

__global__ void k_scatter(int64_t nL, const int32_t *__restrict__ l2g,
                          const double *__restrict__ vG, double *__restrict__ vL) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nL) vL[l] = vG[l2g[l]];
}

__global__ void k_unmask(int64_t nG, const uint8_t *__restrict__ gmask,
                         double *__restrict__ o64, float *__restrict__ o32) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nG) {
    o64[g] = gmask[g] ? 0.0 : 1.0;
    o32[g] = gmask[g] ? 0.0f : 1.0f;
  }
}

// --------------------------------------------------------------------------
// host orchestration
// --------------------------------------------------------------------------
static unsigned nblk(int64_t n) { return (unsigned)((n + RT - 1) / RT); }

struct Workspace {
  DevBuf x64, r64, z64, p64, w64, b64, wL64;
  DevBuf b32, x32, r32, z32, p32, w32, wL32;
  DevBuf one64, one32;       // preconditioner "none": 1 off the boundary
  DevBuf part, st, red;      // partials, CgState, reduce outputs
  CgState *host_st = nullptr;  // pinned
  double *host_red = nullptr;  // pinned
  hipStream_t hs = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, fence = nullptr;
  struct GraphEntry {
    int prec, f32, k, jac;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  ~Workspace() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (host_st) (void)hipHostFree(host_st);
    if (host_red) (void)hipHostFree(host_red);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (fence) (void)hipEventDestroy(fence);
    if (hs) (void)hipStreamDestroy(hs);
  }
};

Workspace *get_ws(sem_handle *h);

struct CgPlan {
  int prec_ax;  // operator precision
  bool f32;     // FP32 vectors
  void *x, *r, *z, *p, *wG, *wL;
  const void *b, *dinv, *G, *D;
};

static void launch_iteration(sem_handle *h, Workspace *W, const CgPlan &P,
                             hipStream_t s) {
  const int nb = red_blocks(h->nG);
  CgState *st = W->st.as<CgState>();
  double *part = W->part.as<double>();
  const int32_t *stop = &st->done;
  launch_ax(h->N, P.prec_ax, h->E, P.D, P.G, P.p, P.wL, h->l2g.as<int32_t>(),
            stop, s);
  if (!P.f32) {
    hipLaunchKernelGGL((k_assemble<double, double, true>), dim3(nb), dim3(RT), 0,
                       s, h->nG, h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                       h->gmask.as<uint8_t>(), (const double *)P.wL,
                       (double *)P.wG, (const double *)P.p, part, stop);
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(RT), 0, s, st, part, nb);
    hipLaunchKernelGGL((k_update_xr<double, double>), dim3(nb), dim3(RT), 0, s,
                       h->nG, st, (double *)P.x, (double *)P.r,
                       (const double *)P.p, (const double *)P.wG,
                       (const double *)P.dinv, (double *)P.z, part, nb);
    hipLaunchKernelGGL(k_beta, dim3(1), dim3(RT), 0, s, st, part, nb);
    hipLaunchKernelGGL((k_update_p<double>), dim3(nb), dim3(RT), 0, s, h->nG,
                       st, (const double *)P.z, (double *)P.p);
  } else {
    hipLaunchKernelGGL((k_assemble<float, float, true>), dim3(nb), dim3(RT), 0,
                       s, h->nG, h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                       h->gmask.as<uint8_t>(), (const float *)P.wL,
                       (float *)P.wG, (const float *)P.p, part, stop);
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(RT), 0, s, st, part, nb);
    hipLaunchKernelGGL((k_update_xr<float, float>), dim3(nb), dim3(RT), 0, s,
                       h->nG, st, (float *)P.x, (float *)P.r,
                       (const float *)P.p, (const float *)P.wG,
                       (const float *)P.dinv, (float *)P.z, part, nb);
    hipLaunchKernelGGL(k_beta, dim3(1), dim3(RT), 0, s, st, part, nb);
    hipLaunchKernelGGL((k_update_p<float>), dim3(nb), dim3(RT), 0, s, h->nG, st,
                       (const float *)P.z, (float *)P.p);
  }
  SEM_HIP(hipGetLastError());
}

// A x for FP64 unique x into W->w64 (through W->wL64)
static void apply_fp64(sem_handle *h, Workspace *W, const double *x,
                       hipStream_t s) {
  const int nb = red_blocks(h->nG);
  launch_ax(h->N, SEM_FP64, h->E, h->D64.p, h->G64.p, x, W->wL64.p,
            h->l2g.as<int32_t>(), nullptr, s);
  hipLaunchKernelGGL((k_assemble<double, double, false>), dim3(nb), dim3(RT), 0,
                     s, h->nG, h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                     h->gmask.as<uint8_t>(), W->wL64.as<double>(),
                     W->w64.as<double>(), (const double *)nullptr,
                     (double *)nullptr, (const int32_t *)nullptr);
  SEM_HIP(hipGetLastError());
}

// ||b - A x||^2 and ||b||^2 (FP64); r stored in W->r64 when store_r
static void residual_fp64(sem_handle *h, Workspace *W, const double *x,
                          bool store_r, hipStream_t s, double &rr, double &bb) {
  apply_fp64(h, W, x, s);
  const int nb = red_blocks(h->nG);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(RT), 0, s, h->nG,
                     W->b64.as<double>(), W->w64.as<double>(),
                     store_r ? W->r64.as<double>() : (double *)nullptr,
                     W->part.as<double>());
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(RT), 0, s, W->part.as<double>(), nb,
                     W->red.as<double>());
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipMemcpyAsync(W->host_red, W->red.p, 2 * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  rr = W->host_red[0];
  bb = W->host_red[1];
}

static void launch_init(sem_handle *h, Workspace *W, const CgPlan &P, bool x0_zero,
                        double tol2, int maxit, hipStream_t s) {
  const int nb = red_blocks(h->nG);
  double *part = W->part.as<double>();
  if (!P.f32) {
    const double *w = nullptr;
    if (!x0_zero) {
      apply_fp64(h, W, (const double *)P.x, s);
      w = W->w64.as<double>();
    }
    hipLaunchKernelGGL((k_init<double, double>), dim3(nb), dim3(RT), 0, s, h->nG,
                       (const double *)P.b, w, (double *)P.x, (double *)P.r,
                       (double *)P.z, (double *)P.p, (const double *)P.dinv,
                       part, nb);
  } else {
    if (!x0_zero) fail(SEM_ERR_STATE, "internal: FP32 CG needs x0 = 0");
    hipLaunchKernelGGL((k_init<float, float>), dim3(nb), dim3(RT), 0, s, h->nG,
                       (const float *)P.b, (const float *)nullptr, (float *)P.x,
                       (float *)P.r, (float *)P.z, (float *)P.p,
                       (const float *)P.dinv, part, nb);
  }
  hipLaunchKernelGGL(k_init_reduce, dim3(1), dim3(RT), 0, s, W->st.as<CgState>(),
                     part, nb, tol2, maxit);
  SEM_HIP(hipGetLastError());
}

static hipGraphExec_t get_graph(sem_handle *h, Workspace *W, const CgPlan &P,
                                int K, int jac, hipStream_t s) {
  for (auto &g : W->graphs)
    if (g.prec == P.prec_ax && g.f32 == (int)P.f32 && g.k == K && g.jac == jac)
      return g.exec;
  hipGraph_t graph;
  SEM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  try {
    for (int q = 0; q < K; ++q) launch_iteration(h, W, P, s);
  } catch (...) {
    hipGraph_t dummy;
    (void)hipStreamEndCapture(s, &dummy);
    throw;
  }
  SEM_HIP(hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec;
  SEM_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  SEM_HIP(hipGraphDestroy(graph));
  W->graphs.push_back({P.prec_ax, (int)P.f32, K, jac, exec});
  return exec;
}

// run CG iterations from an initialised state; returns iterations and the
// device 'done' code
static void run_cg(sem_handle *h, Workspace *W, const CgPlan &P,
                   const sem_solve_opts *o, int jac, hipStream_t s, int &iters,
                   int &done) {
  const int K = std::max(1, o->check_every);
  SEM_HIP(hipMemcpyAsync(W->host_st, W->st.p, sizeof(CgState),
                         hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  while (W->host_st->done == 0) {
    if (o->use_graph) {
      hipGraphExec_t ex = get_graph(h, W, P, K, jac, s);
      SEM_HIP(hipGraphLaunch(ex, s));
    } else {
      for (int q = 0; q < K; ++q) launch_iteration(h, W, P, s);
    }
    SEM_HIP(hipMemcpyAsync(W->host_st, W->st.p, sizeof(CgState),
                           hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
  }
  iters = W->host_st->it;
  done = W->host_st->done;
}

static void ensure_ws(sem_handle *h, Workspace *W) {
  if (W->hs != nullptr) return;
  const size_t g8 = h->nG * sizeof(double), g4 = h->nG * sizeof(float);
  W->x64.alloc(g8);
  W->r64.alloc(g8);
  W->z64.alloc(g8);
  W->p64.alloc(g8);
  W->w64.alloc(g8);
  W->b64.alloc(g8);
  W->wL64.alloc(h->nL * sizeof(double));
  W->b32.alloc(g4);
  W->x32.alloc(g4);
  W->r32.alloc(g4);
  W->z32.alloc(g4);
  W->p32.alloc(g4);
  W->w32.alloc(g4);
  W->wL32.alloc(h->nL * sizeof(float));
  W->one64.alloc(g8);
  W->one32.alloc(g4);
  W->part.alloc(3 * RBLK_MAX * sizeof(double));
  W->st.alloc(sizeof(CgState));
  W->red.alloc(4 * sizeof(double));
  SEM_HIP(hipHostMalloc((void **)&W->host_st, sizeof(CgState), 0));
  SEM_HIP(hipHostMalloc((void **)&W->host_red, 4 * sizeof(double), 0));
  SEM_HIP(hipEventCreate(&W->ev0));
  SEM_HIP(hipEventCreate(&W->ev1));
  SEM_HIP(hipEventCreateWithFlags(&W->fence, hipEventDisableTiming));
  hipStream_t hs;
  SEM_HIP(hipStreamCreateWithFlags(&hs, hipStreamNonBlocking));
  W->hs = hs;
  hipLaunchKernelGGL(k_unmask, dim3(nblk(h->nG)), dim3(RT), 0, hs, h->nG,
                     h->gmask.as<uint8_t>(), W->one64.as<double>(),
                     W->one32.as<float>());
  SEM_HIP(hipGetLastError());
}

sem_status pcg_solve(sem_handle *h, const sem_solve_opts *o, const double *b_L,
                     double *x_L, sem_solve_stats *st, hipStream_t caller) {
  if (!(o->rtol > 0.0) || o->maxit < 0 || o->check_every < 1)
    fail(SEM_ERR_ARG, "sem_pcg_solve: need rtol > 0, maxit >= 0, check_every >= 1");
  if (o->pc != SEM_PC_NONE && o->pc != SEM_PC_JACOBI)
    fail(SEM_ERR_ARG, "sem_pcg_solve: unknown preconditioner");
  if (o->inner_prec != SEM_FP64 && o->inner_prec != SEM_FP32 &&
      o->inner_prec != SEM_BF16)
    fail(SEM_ERR_ARG, "sem_pcg_solve: unknown inner precision");
  if (o->inner_prec != SEM_FP64 && !(o->inner_rtol > 0.0 && o->inner_rtol < 1.0))
    fail(SEM_ERR_ARG, "sem_pcg_solve: inner_rtol must be in (0, 1)");
  Workspace *W = get_ws(h);
  ensure_ws(h, W);
  hipStream_t s = W->hs;
  // order after the caller's stream
  SEM_HIP(hipEventRecord(W->fence, caller));
  SEM_HIP(hipStreamWaitEvent(s, W->fence, 0));
  SEM_HIP(hipEventRecord(W->ev0, s));

  const int jac = o->pc == SEM_PC_JACOBI;
  const int T = RT;
  hipLaunchKernelGGL(k_first_copy, dim3(nblk(h->nG)), dim3(T), 0, s, h->nG,
                     h->offsets.as<int32_t>(), h->perm.as<int32_t>(), b_L,
                     W->b64.as<double>());
  hipLaunchKernelGGL(k_first_copy, dim3(nblk(h->nG)), dim3(T), 0, s, h->nG,
                     h->offsets.as<int32_t>(), h->perm.as<int32_t>(), x_L,
                     W->x64.as<double>());
  SEM_HIP(hipGetLastError());

  int iters = 0, outer = 0, done = 0;
  sem_status status = SEM_OK;
  if (o->inner_prec == SEM_FP64) {
    CgPlan P{SEM_FP64, false, W->x64.p, W->r64.p, W->z64.p, W->p64.p, W->w64.p,
             W->wL64.p, W->b64.p, jac ? h->dinv_G.p : W->one64.p, h->G64.p,
             h->D64.p};
    launch_init(h, W, P, false, o->rtol * o->rtol, o->maxit, s);
    run_cg(h, W, P, o, jac, s, iters, done);
    status = done == 1 ? SEM_OK
             : done == 2 ? SEM_ERR_BREAKDOWN
                         : SEM_ERR_NOT_CONVERGED;
  } else {
    // FP64 iterative refinement: r = b - A64 x; solve A_lo d = r / ||r|| in
    // FP32 vectors with an FP32 or BF16-stored operator; x += ||r|| d
    CgPlan P{o->inner_prec, true, W->x32.p, W->r32.p, W->z32.p, W->p32.p,
             W->w32.p, W->wL32.p, W->b32.p, jac ? h->dinv_G32.p : W->one32.p,
             o->inner_prec == SEM_FP32 ? h->G32.p : h->G16.p, h->D32.p};
    double rr, bb;
    residual_fp64(h, W, W->x64.as<double>(), true, s, rr, bb);
    double rel_prev = 1e300;
    int stall = 0;
    status = SEM_ERR_NOT_CONVERGED;
    while (true) {
      if (!std::isfinite(rr)) {
        status = SEM_ERR_BREAKDOWN;
        break;
      }
      const double rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
      if (rel <= o->rtol) {
        status = SEM_OK;
        break;
      }
      if (iters >= o->maxit) break;
      stall = rel > 0.9 * rel_prev ? stall + 1 : 0;
      if (stall >= 3) break;
      rel_prev = rel;
      const double nr = std::sqrt(rr);
      hipLaunchKernelGGL(k_scale_cast, dim3(nblk(h->nG)), dim3(T), 0, s, h->nG,
                         W->r64.as<double>(), 1.0 / nr, W->b32.as<float>());
      SEM_HIP(hipGetLastError());
      launch_init(h, W, P, true, o->inner_rtol * o->inner_rtol,
                  o->maxit - iters, s);
      int it_in = 0, done_in = 0;
      run_cg(h, W, P, o, jac, s, it_in, done_in);
      iters += it_in;
      outer += 1;
      if (done_in == 2) {
        status = SEM_ERR_BREAKDOWN;
        break;
      }
      hipLaunchKernelGGL(k_axpy_mixed, dim3(nblk(h->nG)), dim3(T), 0, s, h->nG,
                         W->x64.as<double>(), W->x32.as<float>(), nr);
      SEM_HIP(hipGetLastError());
      residual_fp64(h, W, W->x64.as<double>(), true, s, rr, bb);
    }
  }
  // solution back to the caller's E-vector, true FP64 residual
  hipLaunchKernelGGL(k_scatter, dim3(nblk(h->nL)), dim3(T), 0, s, h->nL,
                     h->l2g.as<int32_t>(), W->x64.as<double>(), x_L);
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipEventRecord(W->ev1, s));
  double rr, bb;
  residual_fp64(h, W, W->x64.as<double>(), false, s, rr, bb);
  float ms = 0.0f;
  SEM_HIP(hipEventElapsedTime(&ms, W->ev0, W->ev1));
  if (st != nullptr) {
    st->iters = iters;
    st->outer_iters = outer;
    st->status = status;
    st->reserved = 0;
    st->final_rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    st->seconds = ms * 1e-3;
  }
  // the caller's stream waits for the solve
  SEM_HIP(hipEventRecord(W->fence, s));
  SEM_HIP(hipStreamWaitEvent(caller, W->fence, 0));
  return status;
}

Workspace *get_ws(sem_handle *h) {
  if (h->ws == nullptr) h->ws = new Workspace();
  return h->ws;
}

void destroy_ws(sem_handle *h) {
  delete h->ws;
  h->ws = nullptr;
}

}  // namespace sem
