// Direct stiffness summation (gather-scatter) and the conversions between
// E-vectors and unique-node vectors (paper section 4.2.1: distinct
// global-local node numbering, after Fischer 1991).
//
// Atomic-free and deterministic: the sorted map (perm, offsets) lists the
// local copies of every global node in ascending local index.  One thread
// per global node loads its offsets, its mask flag, the ids of all its
// copies (at most 8 on a hexahedral mesh) and then all their values at once,
// sums them from +0.0 in the listed order and writes the sum back to every
// copy; a Dirichlet node's copies are set to zero without being read.  A
// node with one copy receives +0.0 + v, the same one-term sum: the value
// itself except that -0.0 becomes +0.0, so only that case is written.
// (Three kernels over separate lists of shared, single-copy and Dirichlet
// nodes, each thread walking its segment one load after the other, took
// 125 us at 32^3, N = 7.)
#include "common.h"
#include "sem_internal.h"

namespace sem {

template <class T> __device__ inline bool same_bits(T a, T b) {
  if constexpr (sizeof(T) == 8)
    return __double_as_longlong(a) == __double_as_longlong(b);
  else
    return __float_as_int(a) == __float_as_int(b);
}

template <class T>
__global__ void __launch_bounds__(256)
    k_gs(int64_t nG, const int32_t *__restrict__ off, const int32_t *__restrict__ perm,
         const uint8_t *__restrict__ gmask, T *__restrict__ v) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= nG) return;
  const int32_t a = off[g], cnt = off[g + 1] - a;
  const bool masked = gmask[g] != 0;
  int32_t id[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) id[q] = q < cnt ? perm[a + q] : 0;
  if (masked) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < cnt) v[id[q]] = T(0);
    return;
  }
  T x[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) x[q] = q < cnt ? v[id[q]] : T(0);
  // absent copies add +0.0, which leaves a sum that starts at +0.0 unchanged
  T acc = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) acc = acc + x[q];
  if (cnt == 1) {
    if (!same_bits(acc, x[0])) v[id[0]] = acc;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < cnt) v[id[q]] = acc;
  }
}

static inline unsigned nblk(int64_t n, int t) {
  return (unsigned)((n + t - 1) / t);
}

void launch_gs(sem_handle *h, int prec, void *v, hipStream_t s) {
  if (h->nG == 0) return;
  if (prec == SEM_FP64)
    hipLaunchKernelGGL(k_gs<double>, dim3(nblk(h->nG, 256)), dim3(256), 0, s, h->nG,
                       h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                       h->gmask.as<uint8_t>(), (double *)v);
  else if (prec == SEM_FP32)
    hipLaunchKernelGGL(k_gs<float>, dim3(nblk(h->nG, 256)), dim3(256), 0, s, h->nG,
                       h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                       h->gmask.as<uint8_t>(), (float *)v);
  else
    fail(SEM_ERR_ARG, "sem_gs: precision must be SEM_FP64 or SEM_FP32");
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
