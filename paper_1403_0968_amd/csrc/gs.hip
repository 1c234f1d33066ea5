// Direct stiffness summation (gather-scatter) and the conversions between
// E-vectors and unique-node vectors (paper section 4.2.1: distinct
// global-local node numbering, after Fischer 1991).
//
// Atomic-free and deterministic: every shared global node owns a contiguous
// segment of a precomputed list of its local copies in ascending local
// index; one thread sums the segment from +0.0 in that order and writes the
// sum back to every copy.  Copies of Dirichlet nodes are zeroed from their
// own list (no reads).  A node with a single unmasked copy receives
// +0.0 + v, the same one-term sum: the value itself, except that -0.0
// becomes +0.0.
#include "common.h"
#include "sem_internal.h"

namespace sem {

template <class T>
__global__ void k_zero_ids(int64_t n, const int32_t *__restrict__ ids,
                           T *__restrict__ v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) v[ids[q]] = T(0);
}

// single-copy nodes: v <- +0.0 + v (a sum of one term from +0.0)
template <class T>
__global__ void k_solo_sum(int64_t n, const int32_t *__restrict__ ids,
                           T *__restrict__ v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) {
    const int32_t l = ids[q];
    v[l] = T(0) + v[l];
  }
}

template <class T>
__global__ void k_seg_sum(int64_t nseg, const int32_t *__restrict__ off,
                          const int32_t *__restrict__ ids, T *__restrict__ v) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int a = off[s], b = off[s + 1];
  T acc = T(0);
  for (int q = a; q < b; ++q) acc = acc + v[ids[q]];
  for (int q = a; q < b; ++q) v[ids[q]] = acc;
}

static inline unsigned nblk(int64_t n, int t) {
  return (unsigned)((n + t - 1) / t);
}

void launch_gs(sem_handle *h, int prec, void *v, hipStream_t s) {
  const int T = 256;
  if (prec == SEM_FP64) {
    if (h->n_seg > 0)
      hipLaunchKernelGGL(k_seg_sum<double>, dim3(nblk(h->n_seg, T)), dim3(T), 0,
                         s, h->n_seg, h->seg_off.as<int32_t>(),
                         h->seg_ids.as<int32_t>(), (double *)v);
    if (h->n_solo > 0)
      hipLaunchKernelGGL(k_solo_sum<double>, dim3(nblk(h->n_solo, T)), dim3(T), 0,
                         s, h->n_solo, h->solo_lids.as<int32_t>(), (double *)v);
    if (h->n_masked > 0)
      hipLaunchKernelGGL(k_zero_ids<double>, dim3(nblk(h->n_masked, T)),
                         dim3(T), 0, s, h->n_masked,
                         h->masked_lids.as<int32_t>(), (double *)v);
  } else if (prec == SEM_FP32) {
    if (h->n_seg > 0)
      hipLaunchKernelGGL(k_seg_sum<float>, dim3(nblk(h->n_seg, T)), dim3(T), 0,
                         s, h->n_seg, h->seg_off.as<int32_t>(),
                         h->seg_ids.as<int32_t>(), (float *)v);
    if (h->n_solo > 0)
      hipLaunchKernelGGL(k_solo_sum<float>, dim3(nblk(h->n_solo, T)), dim3(T), 0,
                         s, h->n_solo, h->solo_lids.as<int32_t>(), (float *)v);
    if (h->n_masked > 0)
      hipLaunchKernelGGL(k_zero_ids<float>, dim3(nblk(h->n_masked, T)),
                         dim3(T), 0, s, h->n_masked,
                         h->masked_lids.as<int32_t>(), (float *)v);
  } else {
    fail(SEM_ERR_ARG, "sem_gs: precision must be SEM_FP64 or SEM_FP32");
  }
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// preconditioner on E-vectors
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_precond_local(int64_t nL, const int32_t *__restrict__ l2g,
                                const double *__restrict__ dinv,
                                const uint8_t *__restrict__ bmask,
                                const T *__restrict__ r, T *__restrict__ z,
                                int jacobi) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  if (jacobi)
    z[l] = (T)(dinv[l2g[l]] * (double)r[l]);
  else
    z[l] = bmask[l] ? T(0) : r[l];
}

void learn_precond_local(sem_handle *h, const double *r, double *z, hipStream_t s);

void launch_precond(sem_handle *h, int pc, int prec, const void *r, void *z,
                    hipStream_t s) {
  const int T = 256;
  if (pc == SEM_PC_LEARNED) {
    if (prec != SEM_FP64)
      fail(SEM_ERR_ARG, "sem_precond_apply: the learned preconditioner takes FP64");
    learn_precond_local(h, (const double *)r, (double *)z, s);
    return;
  }
  if (pc != SEM_PC_NONE && pc != SEM_PC_JACOBI)
    fail(SEM_ERR_ARG, "sem_precond_apply: unknown preconditioner");
  const int jac = pc == SEM_PC_JACOBI;
  if (prec == SEM_FP64)
    hipLaunchKernelGGL(k_precond_local<double>, dim3(nblk(h->nL, T)), dim3(T),
                       0, s, h->nL, h->l2g.as<int32_t>(), h->dinv_G.as<double>(),
                       h->bmask.as<uint8_t>(), (const double *)r, (double *)z,
                       jac);
  else if (prec == SEM_FP32)
    hipLaunchKernelGGL(k_precond_local<float>, dim3(nblk(h->nL, T)), dim3(T),
                       0, s, h->nL, h->l2g.as<int32_t>(), h->dinv_G.as<double>(),
                       h->bmask.as<uint8_t>(), (const float *)r, (float *)z,
                       jac);
  else
    fail(SEM_ERR_ARG, "sem_precond_apply: precision must be FP64 or FP32");
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// right-hand side b = mask o Q Q^T (B o f(X))
// ---------------------------------------------------------------------------
struct SrcParams {
  int kind, nmodes;
  double k[64][3], a[64], phi[64];
};

__global__ void k_rhs_local(int64_t nL, const double *__restrict__ X,
                            const double *__restrict__ B, SrcParams p,
                            double *__restrict__ b) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  const double x = X[l], y = X[nL + l], z = X[2 * nL + l];
  const double pi = 3.14159265358979323846;
  double f = 0.0;
  if (p.kind == SEM_SRC_SINE) {
    f = 3.0 * pi * pi * sin(pi * x) * sin(pi * y) * sin(pi * z);
  } else {
    for (int m = 0; m < p.nmodes; ++m)
      f += p.a[m] * cos(2.0 * pi * (p.k[m][0] * x + p.k[m][1] * y +
                                   p.k[m][2] * z) + p.phi[m]);
  }
  b[l] = B[l] * f;
}

void launch_rhs(sem_handle *h, const sem_source *src, double *b, hipStream_t s) {
  SrcParams p{};
  p.kind = src->kind;
  p.nmodes = 0;
  if (src->kind == SEM_SRC_FOURIER) {
    if (src->nmodes < 0 || src->nmodes > 64 || (src->nmodes > 0 &&
        (!src->k || !src->a || !src->phi)))
      fail(SEM_ERR_ARG, "sem_rhs: need 0..64 Fourier modes with k, a, phi");
    p.nmodes = src->nmodes;
    for (int m = 0; m < p.nmodes; ++m) {
      for (int d = 0; d < 3; ++d) p.k[m][d] = src->k[3 * m + d];
      p.a[m] = src->a[m];
      p.phi[m] = src->phi[m];
    }
  } else if (src->kind != SEM_SRC_SINE) {
    fail(SEM_ERR_ARG, "sem_rhs: unknown source kind");
  }
  const int T = 256;
  hipLaunchKernelGGL(k_rhs_local, dim3(nblk(h->nL, T)), dim3(T), 0, s, h->nL,
                     h->coords.as<double>(), h->mass.as<double>(), p, b);
  SEM_HIP(hipGetLastError());
  launch_gs(h, SEM_FP64, b, s);
}

}  // namespace sem
