// Learned per-element correction on a mesh: element features of a
// residual, the network's outputs turned into nodal corrections, and the
// generation of training pairs from FP64 solves followed by GPU training.
//
// Three output layouts, fixed by the network's shape (n3 = (N+1)^3,
// ni = (N-1)^3):
//   Q1       n_in = n3 + 8, n_out = 8: trilinear vertex values prolonged to
//            the GLL nodes; targets from the global error;
//   nodal    n_in = n3 + 8, n_out = n3: one value per node; targets from the
//            global error;
//   interior n_in = ni + 8, n_out = ni: one value per element-interior node
//            (1 <= i, j, k <= N-1); targets from the element-interior solve.
// Features of element e (residual r on unique nodes): r_f = r at the
// feature nodes (all nodes, or the interior ones), s_e = ||r_f||_2,
// x = [r_f / s_e, log kappa at the 8 vertices minus their mean, 0 ...].
// Correction: c_e = s_e / (kappa_e h_e) y_e, with y_e the network output on
// the element's nodes (prolonged, nodal, or interior with zero faces),
// kappa_e the mean of the vertex values and h_e the element size; the solver
// averages c over the copies of every node (interior nodes have one).
// Targets, scaled by kappa_e h_e / s_e so that input and target are O(1):
//   global error: the element error x* - x_k of a snapshot;
//   interior: d - dinv r_I, with d the solution of the element's interior
//   problem A_II d = r_I (the element stiffness with zero values on the
//   element's faces), so that z = dinv r + c is the element-interior block
//   solve wherever the network is exact.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <random>
#include <vector>

#include "ax_tile.h"

namespace sem {

enum { LM_Q1 = 0, LM_NODAL = 1, LM_INTERIOR = 2 };

struct Learn {
  int ldx = 0, n3 = 0, n_out = 0, ldo = 0;
  int mode = LM_NODAL, nf = 0, nt = 0;  // layout, feature nodes, target width
  DevBuf X, s, O, kfeat, invkh, cL, h1, h2;  // h1, h2: hidden activations
};

struct LXi {
  float xi[17];
  int n1;
};

static LXi lxi(const sem_handle *h) {
  LXi p{};
  p.n1 = h->n1;
  for (int q = 0; q < h->n1; ++q) p.xi[q] = (float)h->ref.xi[q];
  return p;
}

// per element: log-kappa vertex features and 1 / (kappa_e h_e)
__global__ void k_kfeat(int64_t E, const double *__restrict__ kv, double h,
                        float *__restrict__ kf, float *__restrict__ invkh) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double lk[8], mean = 0.0, kbar = 0.0;
  for (int v = 0; v < 8; ++v) {
    lk[v] = log(kv[e * 8 + v]);
    mean += lk[v] / 8.0;
    kbar += kv[e * 8 + v] / 8.0;
  }
  for (int v = 0; v < 8; ++v) kf[e * 8 + v] = (float)(lk[v] - mean);
  invkh[e] = (float)(1.0 / (kbar * h));
}

// local index of feature node q: every node, or the element-interior nodes
// 1 <= i, j, k <= N-1 in lexicographic order
__device__ inline int feat_node(int q, int n1, int interior) {
  if (!interior) return q;
  const int m = n1 - 2;
  const int i = q % m, j = (q / m) % m, k = q / (m * m);
  return (i + 1) + n1 * ((j + 1) + n1 * (k + 1));
}

// features of the residual r for every element: r on unique nodes (read
// through l2g) or, with l2g NULL, a continuous E-vector
template <class TV>
__global__ void __launch_bounds__(256)
    k_features(int64_t E, int n1, int interior, int nf,
               const int32_t *__restrict__ l2g, const TV *__restrict__ r,
               const float *__restrict__ kf, uint16_t *__restrict__ X, int ldx,
               float *__restrict__ s) {
  __shared__ double sm[4];
  const int64_t e = blockIdx.x;
  const int n3 = n1 * n1 * n1;
  auto val = [&](int q) -> double {
    const int64_t l = e * n3 + feat_node(q, n1, interior);
    return (double)r[l2g ? (int64_t)l2g[l] : l];
  };
  double ss = 0.0;
  for (int q = threadIdx.x; q < nf; q += 256) {
    const double v = val(q);
    ss += v * v;
  }
  ss = block_sum<256>(ss, sm);
  if (threadIdx.x == 0) sm[0] = ss;
  __syncthreads();
  const double nrm = sqrt(sm[0]);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  uint16_t *xe = X + e * (int64_t)ldx;
  for (int q = threadIdx.x; q < nf; q += 256)
    xe[q] = f32_to_bf16((float)(val(q) * inv));
  if (threadIdx.x < 8) xe[nf + threadIdx.x] = f32_to_bf16(kf[e * 8 + threadIdx.x]);
  if (threadIdx.x == 0) s[e] = (float)nrm;
}

// cL[e][node] = damping s_e invkh_e y(node), with y = sum_v P[node][v] O[e][v]
// (Q1), y = O[e][node] (nodal) or y = O[e][interior index of node] and 0 on
// the element's faces (interior)
__global__ void __launch_bounds__(256)
    k_correct(int64_t E, LXi xp, int mode, const float *__restrict__ O, int ldo,
              const float *__restrict__ s, const float *__restrict__ invkh,
              const float *__restrict__ damping, float *__restrict__ cL) {
  const int64_t e = blockIdx.x;
  const int n1 = xp.n1, n3 = n1 * n1 * n1, N = n1 - 1;
  const float sc = damping[0] * s[e] * invkh[e];
  if (mode == LM_NODAL) {
    for (int p = threadIdx.x; p < n3; p += 256) cL[e * n3 + p] = sc * O[e * ldo + p];
    return;
  }
  if (mode == LM_INTERIOR) {
    const int m = N - 1;
    for (int p = threadIdx.x; p < n3; p += 256) {
      const int i = p % n1, j = (p / n1) % n1, k = p / (n1 * n1);
      const bool in = i > 0 && i < N && j > 0 && j < N && k > 0 && k < N;
      cL[e * n3 + p] =
          in ? sc * O[e * ldo + (i - 1) + m * ((j - 1) + m * (k - 1))] : 0.f;
    }
    return;
  }
  float o[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) o[v] = O[e * ldo + v];
  for (int p = threadIdx.x; p < n3; p += 256) {
    const int i = p % n1, j = (p / n1) % n1, k = p / (n1 * n1);
    const float px[2] = {0.5f * (1.f - xp.xi[i]), 0.5f * (1.f + xp.xi[i])};
    const float py[2] = {0.5f * (1.f - xp.xi[j]), 0.5f * (1.f + xp.xi[j])};
    const float pz[2] = {0.5f * (1.f - xp.xi[k]), 0.5f * (1.f + xp.xi[k])};
    float y = 0.f;
#pragma unroll
    for (int v = 0; v < 8; ++v) y += px[v & 1] * py[(v >> 1) & 1] * pz[v >> 2] * o[v];
    cL[e * n3 + p] = sc * y;
  }
}

static double elem_size(const sem_handle *h) {
  return std::cbrt((1.0 / h->ex) * (1.0 / h->ey) * (1.0 / h->ez));
}

void learn_destroy(sem_handle *h) {
  // (called after the handle's solver state is gone)
  delete h->learn;
  h->learn = nullptr;
  h->net = nullptr;
}

// layout of a network on a mesh (fails when its shape fits none)
static int layout_of(const sem_handle *h, const sem_mlp *net) {
  int n_in = 0, n_out = 0;
  mlp_info(net, &n_in, nullptr, &n_out, nullptr, nullptr);
  const int n3 = h->n1 * h->n1 * h->n1, m = h->N - 1, ni = m * m * m;
  if (n_in == n3 + 8 && n_out == 8) return LM_Q1;
  if (n_in == n3 + 8 && n_out == n3) return LM_NODAL;
  if (ni > 0 && n_in == ni + 8 && n_out == ni) return LM_INTERIOR;
  fail(SEM_ERR_ARG, "learned correction: the network needs n_in = (N+1)^3 + 8 "
                    "and n_out = 8 or (N+1)^3, or n_in = (N-1)^3 + 8 and "
                    "n_out = (N-1)^3 (N >= 2)");
}

static void check_net(const sem_handle *h, const sem_mlp *net) {
  (void)layout_of(h, net);
}

static void kappa_features(const sem_handle *h, DevBuf &kfeat, DevBuf &invkh) {
  kfeat.alloc(h->E * 8 * 4);
  invkh.alloc(h->E * 4);
  hipLaunchKernelGGL(k_kfeat, dim3((unsigned)((h->E + 255) / 256)), dim3(256), 0,
                     0, h->E, h->kvert.as<double>(), elem_size(h),
                     kfeat.as<float>(), invkh.as<float>());
  SEM_HIP(hipGetLastError());
}

static void ensure_learn(sem_handle *h, const sem_mlp *net) {
  const int ldx = mlp_padded_inputs(net);
  const int mode = layout_of(h, net);
  int n_out = 0;
  mlp_info(net, nullptr, nullptr, &n_out, nullptr, nullptr);
  if (h->learn && h->learn->ldx == ldx && h->learn->n_out == n_out &&
      h->learn->mode == mode)
    return;
  delete h->learn;
  h->learn = nullptr;
  Learn *L = new Learn();
  try {
    L->ldx = ldx;
    L->n3 = h->n1 * h->n1 * h->n1;
    L->n_out = n_out;
    L->mode = mode;
    L->nf = mode == LM_INTERIOR ? n_out : L->n3;
    L->nt = mode == LM_INTERIOR ? n_out : L->n3;
    L->ldo = n_out > 16 ? n_out : 16;
    L->X.alloc((size_t)h->E * ldx * 2);
    SEM_HIP(hipMemset(L->X.p, 0, (size_t)h->E * ldx * 2));  // zero padding
    L->s.alloc(h->E * 4);
    L->O.alloc((size_t)h->E * L->ldo * 4);
    L->cL.alloc(h->nL * 4);
    L->h1.alloc((size_t)h->E * 128 * 2);
    L->h2.alloc((size_t)h->E * 128 * 2);
    kappa_features(h, L->kfeat, L->invkh);
    SEM_HIP(hipDeviceSynchronize());
  } catch (...) {
    delete L;
    throw;
  }
  h->learn = L;
}

void drop_graphs(sem_handle *h);

void learn_attach(sem_handle *h, sem_mlp *net) {
  drop_graphs(h);
  if (net == nullptr) {
    h->net = nullptr;
    return;
  }
  check_net(h, net);
  ensure_learn(h, net);
  h->net = net;
}

void learn_apply(sem_handle *h, const void *r, bool f32, float *cL,
                 hipStream_t s) {
  Learn *L = h->learn;
  if (L == nullptr || h->net == nullptr)
    fail(SEM_ERR_STATE, "learned correction: no network attached");
  const int interior = L->mode == LM_INTERIOR;
  if (f32)
    hipLaunchKernelGGL(k_features<float>, dim3((unsigned)h->E), dim3(256), 0, s,
                       h->E, h->n1, interior, L->nf, h->l2g.as<int32_t>(),
                       (const float *)r, L->kfeat.as<float>(), L->X.as<uint16_t>(),
                       L->ldx, L->s.as<float>());
  else
    hipLaunchKernelGGL(k_features<double>, dim3((unsigned)h->E), dim3(256), 0, s,
                       h->E, h->n1, interior, L->nf, h->l2g.as<int32_t>(),
                       (const double *)r, L->kfeat.as<float>(), L->X.as<uint16_t>(),
                       L->ldx, L->s.as<float>());
  SEM_HIP(hipGetLastError());
  mlp_forward(h->net, L->X.as<uint16_t>(), L->ldx, (int)h->E, L->O.as<float>(),
              L->ldo, false, s, L->h1.as<uint16_t>(), L->h2.as<uint16_t>());
  hipLaunchKernelGGL(k_correct, dim3((unsigned)h->E), dim3(256), 0, s, h->E,
                     lxi(h), L->mode, L->O.as<float>(), L->ldo,
                     L->s.as<float>(), L->invkh.as<float>(),
                     mlp_damping_dev(h->net), cL ? cL : L->cL.as<float>());
  SEM_HIP(hipGetLastError());
}

float *learn_cl(sem_handle *h) { return h->learn ? h->learn->cL.as<float>() : nullptr; }

// z_L = dinv o r_L + (average over copies of the correction) on continuous
// E-vectors (FP64), for sem_precond_apply
__global__ void k_precond_learned_local(int64_t nL, const int32_t *__restrict__ l2g,
                                        const int32_t *__restrict__ off,
                                        const int32_t *__restrict__ perm,
                                        const uint8_t *__restrict__ bmask,
                                        const double *__restrict__ dinv,
                                        const float *__restrict__ cL,
                                        const double *__restrict__ r,
                                        double *__restrict__ z) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  if (bmask[l]) {
    z[l] = 0.0;
    return;
  }
  const int64_t g = l2g[l];
  const int a = off[g], b = off[g + 1];
  float c = 0.f;
  for (int k = a; k < b; ++k) c += cL[perm[k]];
  z[l] = dinv[g] * r[l] + (double)(c / (float)(b - a));
}

void learn_precond_local(sem_handle *h, const double *r, double *z, hipStream_t s) {
  Learn *L = h->learn;
  if (L == nullptr || h->net == nullptr)
    fail(SEM_ERR_STATE, "learned correction: no network attached");
  hipLaunchKernelGGL(k_features<double>, dim3((unsigned)h->E), dim3(256), 0, s,
                     h->E, h->n1, L->mode == LM_INTERIOR ? 1 : 0, L->nf,
                     (const int32_t *)nullptr, r, L->kfeat.as<float>(),
                     L->X.as<uint16_t>(), L->ldx, L->s.as<float>());
  SEM_HIP(hipGetLastError());
  mlp_forward(h->net, L->X.as<uint16_t>(), L->ldx, (int)h->E, L->O.as<float>(),
              L->ldo, false, s, L->h1.as<uint16_t>(), L->h2.as<uint16_t>());
  hipLaunchKernelGGL(k_correct, dim3((unsigned)h->E), dim3(256), 0, s, h->E,
                     lxi(h), L->mode, L->O.as<float>(), L->ldo,
                     L->s.as<float>(), L->invkh.as<float>(),
                     mlp_damping_dev(h->net), L->cL.as<float>());
  hipLaunchKernelGGL(k_precond_learned_local, dim3((unsigned)((h->nL + 255) / 256)),
                     dim3(256), 0, s, h->nL, h->l2g.as<int32_t>(),
                     h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                     h->bmask.as<uint8_t>(), h->dinv_G.as<double>(),
                     L->cL.as<float>(), r, z);
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// training pairs and training
// ---------------------------------------------------------------------------
// pair p: features of snapshot residual rs[snap] on element e and target
// (x* - xs[snap]) kappa_e h_e / s_e on the element's nodes
__global__ void __launch_bounds__(256)
    k_build_pairs(int np, const int32_t *__restrict__ psnap,
                  const int32_t *__restrict__ pelem, int64_t nG, int n1,
                  const int32_t *__restrict__ l2g, const double *__restrict__ xs,
                  const double *__restrict__ rs, const double *__restrict__ xstar,
                  const float *__restrict__ kf, const float *__restrict__ invkh,
                  uint16_t *__restrict__ X, int ldx, float *__restrict__ T) {
  __shared__ double sm[4];
  const int p = blockIdx.x;
  if (p >= np) return;
  const int n3 = n1 * n1 * n1;
  const int64_t e = pelem[p];
  const double *r = rs + (int64_t)psnap[p] * nG;
  const double *x = xs + (int64_t)psnap[p] * nG;
  double ss = 0.0;
  for (int q = threadIdx.x; q < n3; q += 256) {
    const double v = r[l2g[e * n3 + q]];
    ss += v * v;
  }
  ss = block_sum<256>(ss, sm);
  if (threadIdx.x == 0) sm[0] = ss;
  __syncthreads();
  const double nrm = sqrt(sm[0]);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  const double tsc = nrm > 0.0 ? 1.0 / (nrm * (double)invkh[e]) : 0.0;
  uint16_t *xp = X + (int64_t)p * ldx;
  float *tp = T + (int64_t)p * n3;
  for (int q = threadIdx.x; q < n3; q += 256) {
    const int64_t g = l2g[e * n3 + q];
    xp[q] = f32_to_bf16((float)(r[g] * inv));
    tp[q] = (float)((xstar[g] - x[g]) * tsc);
  }
  if (threadIdx.x < 8) xp[n3 + threadIdx.x] = f32_to_bf16(kf[e * 8 + threadIdx.x]);
}

__global__ void k_gather_rows(int B, const int32_t *__restrict__ idx,
                              const uint16_t *__restrict__ X, int ldx,
                              const float *__restrict__ T, int n3,
                              uint16_t *__restrict__ Xb, float *__restrict__ Tb) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const int64_t src = idx[b];
  for (int q = threadIdx.x; q < ldx; q += blockDim.x)
    Xb[(int64_t)b * ldx + q] = X[src * ldx + q];
  for (int q = threadIdx.x; q < n3; q += blockDim.x)
    Tb[(int64_t)b * n3 + q] = T[src * n3 + q];
}

// sum over the workgroup, returned to every thread (fixed order: the wave
// butterfly leaves identical bits in every lane, then the waves in order)
template <int NT>
__device__ inline double block_allsum(double v, double *red /* NT / 64 */) {
  v = wave_sum(v);
  if constexpr (NT == 64) return v;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();  // earlier readers of red are done
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) t += red[q];
  return t;
}

// Pairs of the interior layout, one workgroup per pair p: residual r (a
// snapshot rs[psnap[p]] on unique nodes read through l2g, or, with
// local_r, the continuous E-vector rs) restricted to the interior nodes of
// element pelem[p].  Features X[p] = [r_I / s, log kappa deviations] and
// target T[p] = (d - dinv r_I) kappa_e h_e / s, where d solves the
// element's interior problem A_II d = r_I by Jacobi-preconditioned CG
// inside the workgroup: the element operator (the shared element routine,
// zero values on the element's faces) through the pair's scratch rows U, W,
// vectors of a column in the registers of its thread, FP64 throughout,
// stopping at ||r_I - A_II d|| <= rtol ||r_I|| or after maxit iterations.
template <int N1, int NT>
__global__ void __launch_bounds__(NT)
    k_interior_pairs(int np, const int32_t *__restrict__ psnap,
                     const int32_t *__restrict__ pelem, int64_t nG, int local_r,
                     const int32_t *__restrict__ l2g, const double *__restrict__ rs,
                     const double *__restrict__ dinvG, const double *__restrict__ G,
                     const double *__restrict__ D, const float *__restrict__ kf,
                     const float *__restrict__ invkh, uint16_t *__restrict__ X,
                     int ldx, float *__restrict__ T, double *__restrict__ U,
                     double *__restrict__ W, int maxit, double rtol,
                     int32_t *__restrict__ iters) {
  constexpr int NP = N1 * N1, N3 = NP * N1, N = N1 - 1, M = N1 - 2;
  constexpr int NI = M * M * M;
  __shared__ double smem[lds_words<N1>(1)];
  __shared__ double red[NT / 64];
  const int p = blockIdx.x;
  if (p >= np) return;  // uniform per block
  const int t = threadIdx.x;
  const bool act = t < NP;
  const int c = act ? t : 0;
  const int i = c % N1, j = c / N1;
  const bool colI = act && i > 0 && i < N && j > 0 && j < N;
  const int64_t e = pelem[p];
  const double *r = local_r ? rs : rs + (int64_t)psnap[p] * nG;
  double b[N1], dv[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const bool in = colI && k > 0 && k < N;
    const int64_t l = e * N3 + c + k * NP;
    const int64_t g = in ? (int64_t)l2g[l] : 0;
    b[k] = in ? r[local_r ? l : g] : 0.0;
    dv[k] = in ? dinvG[g] : 0.0;
  }
  double ss = 0.0;
#pragma unroll
  for (int k = 0; k < N1; ++k) ss += b[k] * b[k];
  ss = block_allsum<NT>(ss, red);
  const double nrm = sqrt(ss);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  uint16_t *xe = X + (int64_t)p * ldx;
  float *te = T + (int64_t)p * NI;
#pragma unroll
  for (int k = 1; k < N; ++k)
    if (colI) xe[(i - 1) + M * ((j - 1) + M * (k - 1))] = f32_to_bf16((float)(b[k] * inv));
  if (t < 8) xe[NI + t] = f32_to_bf16(kf[e * 8 + t]);

  double x[N1], rr[N1], pp[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    x[k] = 0.0;
    rr[k] = b[k];
    pp[k] = dv[k] * b[k];
  }
  double rz = 0.0;
#pragma unroll
  for (int k = 0; k < N1; ++k) rz += rr[k] * pp[k];
  rz = block_allsum<NT>(rz, red);
  double *u = U + (int64_t)p * N3;
  double *w = W + (int64_t)p * N3;
  const double *Ge = G + e * 6 * N3;
  const double stop2 = rtol * rtol * ss;
  double rn2 = ss;
  int it = 0;
  while (it < maxit && rn2 > stop2) {  // uniform: reduced values
#pragma unroll
    for (int k = 0; k < N1; ++k)
      if (act) u[c + k * NP] = pp[k];
    // the element routine reads and writes the column of this thread
    ax_tile<N1, 1, double, double, double, double, false, false>(
        t, 0, 1, D, Ge, u, w, nullptr, smem);
    double q[N1], pq = 0.0;
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      q[k] = (colI && k > 0 && k < N) ? w[c + k * NP] : 0.0;
      pq += pp[k] * q[k];
    }
    pq = block_allsum<NT>(pq, red);
    if (!(pq > 0.0)) break;
    const double alpha = rz / pq;
    double a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      x[k] += alpha * pp[k];
      rr[k] -= alpha * q[k];
      a2 += rr[k] * rr[k];
      a3 += rr[k] * dv[k] * rr[k];
    }
    rn2 = block_allsum<NT>(a2, red);
    const double rzn = block_allsum<NT>(a3, red);
    const double beta = rzn / rz;
    rz = rzn;
#pragma unroll
    for (int k = 0; k < N1; ++k) pp[k] = dv[k] * rr[k] + beta * pp[k];
    ++it;
  }
  const double tsc = nrm > 0.0 ? 1.0 / (nrm * (double)invkh[e]) : 0.0;
#pragma unroll
  for (int k = 1; k < N; ++k)
    if (colI)
      te[(i - 1) + M * ((j - 1) + M * (k - 1))] =
          (float)((x[k] - dv[k] * b[k]) * tsc);
  if (t == 0 && iters) iters[p] = it;
}

template <int N1>
static void launch_pairs_n(const sem_handle *h, int np, const int32_t *psnap,
                           const int32_t *pelem, int local_r, const double *rs,
                           const float *kf, const float *invkh, uint16_t *X,
                           int ldx, float *T, double *U, double *W, int maxit,
                           double rtol, int32_t *iters, hipStream_t s) {
  constexpr int NT = N1 * N1 <= 64 ? 64 : 128;
  hipLaunchKernelGGL((k_interior_pairs<N1, NT>), dim3(np), dim3(NT), 0, s, np,
                     psnap, pelem, h->nG, local_r, h->l2g.as<int32_t>(), rs,
                     h->dinv_G.as<double>(), h->G64.as<double>(),
                     h->D64.as<double>(), kf, invkh, X, ldx, T, U, W, maxit, rtol,
                     iters);
}

// interior pairs for np (snapshot, element) pairs; U, W: np (N+1)^3 doubles
static void launch_interior_pairs(const sem_handle *h, int np,
                                  const int32_t *psnap, const int32_t *pelem,
                                  int local_r, const double *rs, const float *kf,
                                  const float *invkh, uint16_t *X, int ldx,
                                  float *T, double *U, double *W, int maxit,
                                  double rtol, int32_t *iters, hipStream_t s) {
  if (np <= 0) return;
  switch (h->N) {
#define SEM_PAIRS(NN)                                                          \
  case NN:                                                                     \
    launch_pairs_n<NN + 1>(h, np, psnap, pelem, local_r, rs, kf, invkh, X, ldx, \
                           T, U, W, maxit, rtol, iters, s);                    \
    break;
    SEM_PAIRS(2)
    SEM_PAIRS(3)
    SEM_PAIRS(4)
    SEM_PAIRS(5)
    SEM_PAIRS(6)
    SEM_PAIRS(7)
    SEM_PAIRS(8)
#undef SEM_PAIRS
    default:
      fail(SEM_ERR_ARG, "interior pairs: N must be in 2..8");
  }
  SEM_HIP(hipGetLastError());
}

constexpr int LOCAL_MAXIT = 2000;     // element-interior CG iteration cap
constexpr double LOCAL_RTOL = 1e-10;  // element-interior CG tolerance

void learn_interior_pairs(sem_handle *h, const double *rL, const int32_t *elems,
                          int n, uint16_t *X, int ldx, float *T, double rtol,
                          int32_t *iters, hipStream_t s) {
  const int m = h->N - 1;
  if (m < 1) fail(SEM_ERR_ARG, "interior pairs: N must be at least 2");
  if (n < 0 || (n > 0 && (!rL || !elems || !X || !T)))
    fail(SEM_ERR_ARG, "interior pairs: null argument");
  if (ldx < m * m * m + 8 || ldx % 16 != 0)
    fail(SEM_ERR_ARG, "interior pairs: ldx must be a multiple of 16 and at "
                      "least (N-1)^3 + 8");
  if (!(rtol > 0.0)) fail(SEM_ERR_ARG, "interior pairs: rtol must be positive");
  if (n == 0) return;
  std::vector<int32_t> he(n);
  SEM_HIP(hipMemcpy(he.data(), elems, (size_t)n * 4, hipMemcpyDeviceToHost));
  for (int q = 0; q < n; ++q)
    if (he[q] < 0 || he[q] >= h->E)
      fail(SEM_ERR_ARG, "interior pairs: element index out of range");
  DevBuf kf, ik, U, W;
  kappa_features(h, kf, ik);
  U.alloc((size_t)n * h->n1 * h->n1 * h->n1 * 8);
  W.alloc((size_t)n * h->n1 * h->n1 * h->n1 * 8);
  launch_interior_pairs(h, n, nullptr, elems, 1, rL, kf.as<float>(),
                        ik.as<float>(), X, ldx, T, U.as<double>(), W.as<double>(),
                        LOCAL_MAXIT, rtol, iters, s);
  SEM_HIP(hipStreamSynchronize(s));
}

// snapshot-recording FP64 Jacobi-PCG (solver.hip)
int solve_with_snapshots(sem_handle *h, const double *bL, double *xL, double rtol,
                         int every, int max_snaps, double *xs, double *rs,
                         int *iters, hipStream_t caller);
const double *solution_vector(sem_handle *h);

void learn_train(sem_handle *h, sem_mlp *net, const double *const *bL, int nrhs,
                 const sem_train_opts *o, sem_train_report *rep,
                 hipStream_t caller) {
  check_net(h, net);
  if (nrhs < 1 || bL == nullptr) fail(SEM_ERR_ARG, "train: need right-hand sides");
  if (o->n_pairs < 1 || o->snapshot_every < 1 || o->max_snapshots < 1 ||
      o->epochs < 1 || o->batch < 1 || !(o->lr > 0) || !(o->solve_rtol > 0))
    fail(SEM_ERR_ARG, "train: invalid options");
  ensure_learn(h, net);
  Learn *L = h->learn;
  const int n3 = L->n3, ldx = L->ldx;
  const int64_t nG = h->nG;
  auto t0 = std::chrono::steady_clock::now();

  DevBuf xs, rs, xL, Xd, Td, ps, pe, Xb, Tb, idx;
  xs.alloc((size_t)o->max_snapshots * nG * 8);
  rs.alloc((size_t)o->max_snapshots * nG * 8);
  xL.alloc(h->nL * 8);
  Xd.alloc((size_t)o->n_pairs * ldx * 2);
  SEM_HIP(hipMemset(Xd.p, 0, (size_t)o->n_pairs * ldx * 2));
  const int nt = L->nt;
  const bool interior = L->mode == LM_INTERIOR;
  Td.alloc((size_t)o->n_pairs * nt * 4);
  DevBuf U, W, litn;
  int local_max = 0;
  ps.alloc((size_t)o->n_pairs * 4);
  pe.alloc((size_t)o->n_pairs * 4);
  std::mt19937_64 rng(o->seed);
  int built = 0, total_snaps = 0;
  double rate_sum = 0.0;
  int rate_n = 0;
  for (int q = 0; q < nrhs; ++q) {
    const int want = o->n_pairs / nrhs + (q == nrhs - 1 ? o->n_pairs % nrhs : 0);
    SEM_HIP(hipMemset(xL.p, 0, h->nL * 8));
    int its = 0;
    const int ns = solve_with_snapshots(h, bL[q], xL.as<double>(), o->solve_rtol,
                                        o->snapshot_every, o->max_snapshots,
                                        xs.as<double>(), rs.as<double>(), &its,
                                        caller);
    total_snaps += ns;
    if (its > 0) {
      rate_sum += std::log10(o->solve_rtol) / its;
      rate_n += 1;
    }
    if (ns == 0 || want == 0) continue;
    std::vector<int32_t> hs(want), he(want);
    for (int p = 0; p < want; ++p) {
      hs[p] = (int32_t)(rng() % (uint64_t)ns);
      he[p] = (int32_t)(rng() % (uint64_t)h->E);
    }
    SEM_HIP(hipMemcpy(ps.p, hs.data(), want * 4, hipMemcpyHostToDevice));
    SEM_HIP(hipMemcpy(pe.p, he.data(), want * 4, hipMemcpyHostToDevice));
    if (interior) {
      if (U.p == nullptr) {
        const size_t rows = (size_t)(o->n_pairs / nrhs + o->n_pairs % nrhs);
        U.alloc(rows * n3 * 8);
        W.alloc(rows * n3 * 8);
        litn.alloc(rows * 4);
      }
      launch_interior_pairs(h, want, ps.as<int32_t>(), pe.as<int32_t>(), 0,
                            rs.as<double>(), L->kfeat.as<float>(),
                            L->invkh.as<float>(),
                            Xd.as<uint16_t>() + (int64_t)built * ldx, ldx,
                            Td.as<float>() + (int64_t)built * nt, U.as<double>(),
                            W.as<double>(), LOCAL_MAXIT, LOCAL_RTOL,
                            litn.as<int32_t>(), 0);
      std::vector<int32_t> hi(want);
      SEM_HIP(hipMemcpy(hi.data(), litn.p, (size_t)want * 4, hipMemcpyDeviceToHost));
      for (int v : hi) local_max = std::max(local_max, v);
    } else {
      hipLaunchKernelGGL(k_build_pairs, dim3(want), dim3(256), 0, 0, want,
                         ps.as<int32_t>(), pe.as<int32_t>(), nG, h->n1,
                         h->l2g.as<int32_t>(), xs.as<double>(), rs.as<double>(),
                         solution_vector(h), L->kfeat.as<float>(),
                         L->invkh.as<float>(),
                         Xd.as<uint16_t>() + (int64_t)built * ldx, ldx,
                         Td.as<float>() + (int64_t)built * n3);
      SEM_HIP(hipGetLastError());
    }
    SEM_HIP(hipDeviceSynchronize());
    built += want;
  }
  auto t1 = std::chrono::steady_clock::now();
  if (built == 0) fail(SEM_ERR_STATE, "train: no training pairs were generated");

  const int B = std::min(o->batch, built);
  Xb.alloc((size_t)B * ldx * 2);
  Tb.alloc((size_t)B * nt * 4);
  idx.alloc((size_t)built * 4);
  std::vector<int32_t> perm(built);
  double first = 0.0, last = 0.0;
  hipStream_t s = nullptr;
  for (int ep = 0; ep < o->epochs; ++ep) {
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    SEM_HIP(hipMemcpy(idx.p, perm.data(), built * 4, hipMemcpyHostToDevice));
    double sum = 0.0;
    int nb = 0;
    for (int b0 = 0; b0 + B <= built; b0 += B) {
      hipLaunchKernelGGL(k_gather_rows, dim3(B), dim3(256), 0, s, B,
                         idx.as<int32_t>() + b0, Xd.as<uint16_t>(), ldx,
                         Td.as<float>(), nt, Xb.as<uint16_t>(), Tb.as<float>());
      SEM_HIP(hipGetLastError());
      sum += mlp_loss_grad(net, Xb.as<uint16_t>(), ldx, Tb.as<float>(), B, h->N,
                           true, s);
      mlp_adam(net, nullptr, o->lr, 0.9, 0.999, 1e-8, s);
      ++nb;
    }
    const double mean = nb ? sum / nb : 0.0;
    if (ep == 0) first = mean;
    last = mean;
  }
  SEM_HIP(hipDeviceSynchronize());
  auto t2 = std::chrono::steady_clock::now();

  // Damping of the correction: the learned flexible-CG solve of the last
  // training right-hand side to 1e-6 is compared with Jacobi-PCG for a few
  // damping values (around 1 for the interior layout, whose exact network
  // reproduces the element-interior solve; small for the global-error
  // layouts); the best one is kept if it needs fewer iterations than
  // Jacobi, else the correction is disabled (damping 0).
  sem_mlp *prev = h->net;
  const double rate = rate_n ? rate_sum / rate_n : 0.0;
  mlp_set_damping(net, 1.0, 0.0);  // no progress judge while validating
  learn_attach(h, net);
  sem_solve_opts vo{};
  vo.rtol = 1e-6;
  vo.maxit = 100000;
  vo.pc = SEM_PC_JACOBI;
  vo.inner_prec = SEM_FP64;
  vo.inner_rtol = 0.1;
  vo.check_every = 8;
  vo.use_graph = 1;
  sem_solve_stats vs{};
  SEM_HIP(hipMemset(xL.p, 0, h->nL * 8));
  pcg_solve(h, &vo, bL[nrhs - 1], xL.as<double>(), &vs, caller);
  const int it_jac = vs.iters;
  const double cand_int[4] = {1.0, 0.75, 0.5, 0.25};
  const double cand_glob[4] = {0.2, 0.15, 0.1, 0.05};
  const double *cand = interior ? cand_int : cand_glob;
  double best_d = 0.0;
  int best_it = it_jac;
  int cand_it[4] = {-1, -1, -1, -1};
  vo.pc = SEM_PC_LEARNED;
  vo.maxit = 2 * it_jac + 10;
  for (int c = 0; c < 4; ++c) {
    const double d = cand[c];
    mlp_set_damping(net, d, 0.0);
    SEM_HIP(hipMemset(xL.p, 0, h->nL * 8));
    const sem_status st = pcg_solve(h, &vo, bL[nrhs - 1], xL.as<double>(), &vs, caller);
    if (st == SEM_OK && vs.fell_back == 0) {
      cand_it[c] = vs.iters;
      if (vs.iters < best_it) {
        best_it = vs.iters;
        best_d = d;
      }
    }
  }
  mlp_set_damping(net, best_d, rate);
  learn_attach(h, prev);
  auto t3 = std::chrono::steady_clock::now();
  if (rep) {
    rep->pairs = built;
    rep->epochs = o->epochs;
    rep->snapshots = total_snaps;
    rep->local_iters_max = local_max;
    rep->first_loss = first;
    rep->last_loss = last;
    rep->data_seconds = std::chrono::duration<double>(t1 - t0).count();
    rep->train_seconds = std::chrono::duration<double>(t2 - t1).count();
    rep->damping = best_d;
    rep->val_iters_jacobi = it_jac;
    rep->val_iters_learned = best_d > 0 ? best_it : it_jac;
    rep->validate_seconds = std::chrono::duration<double>(t3 - t2).count();
    rep->jacobi_rate = rate;
    for (int c = 0; c < 4; ++c) rep->val_iters[c] = cand_it[c];
  }
}

}  // namespace sem
