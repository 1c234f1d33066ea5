// Direct stiffness summation (gather-scatter) and the conversions between
// E-vectors and unique-node vectors (paper section 4.2.1: distinct
// global-local node numbering, after Fischer 1991).
//
// Atomic-free and deterministic.  A thread per global node enumerates the
// node's local copies (at most 8 on a hexahedral mesh) in closed form from
// the node's box coordinates, loads all their values at once, sums them
// from +0.0 in ascending local index (the order of the sorted map perm /
// offsets that the exports hold) and writes the sum back to every copy; a
// Dirichlet node's copies are set to zero without being read.  A node with
// one copy receives +0.0 + v, the same one-term sum: the value itself
// except that -0.0 becomes +0.0, so only that case is written.  (Reading
// the copies' ids from the sorted map took 90 us at 32^3, N = 7; three
// kernels over separate lists of shared, single-copy and Dirichlet nodes,
// each thread walking its segment one load after the other, 125 us.)
#include "common.h"
#include "sem_internal.h"

#include <type_traits>

namespace sem {

template <class T> __device__ inline bool same_bits(T a, T b) {
  if constexpr (sizeof(T) == 8)
    return __double_as_longlong(a) == __double_as_longlong(b);
  else
    return __float_as_int(a) == __float_as_int(b);
}

// The copies' local indices come from the per-direction terms of
// structured.h, so the kernel moves only the E-vector.  GS_K nodes per
// thread, GS_T apart (coordinates advanced by carries), all their copies
// loaded before any sum is formed.
constexpr int GS_T = 256, GS_K = 2;  // 1: 68 us, 2: 61 us, 4: 75 us (FP64, 32^3, N = 7)

template <class T, bool PER, bool W64>
__global__ void __launch_bounds__(GS_T) k_gs_box(Box bx, int64_t nG, T *__restrict__ v_) {
  const gp<T> v = (gp<T>)v_;
  using IT = typename std::conditional<W64, int64_t, uint32_t>::type;
  const int64_t g0 = (int64_t)blockIdx.x * (GS_T * GS_K) + threadIdx.x;
  Coord3 pc = box_coord(bx, (uint32_t)g0);
  const Coord3 step = box_coord(bx, (uint32_t)GS_T);
  IT lid[GS_K][8];
  T x[GS_K][8];
  bool live[GS_K][8], masked[GS_K];
  int cnt[GS_K];
#pragma unroll
  for (int k = 0; k < GS_K; ++k) {
    const bool act = g0 + k * GS_T < nG;
    const CopyTerms<IT> ct = copy_terms<IT, PER>(bx, pc);
    masked[k] = ct.masked;
    cnt[k] = ct.x.cnt * ct.y.cnt * ct.z.cnt;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int q = 4 * a + 2 * b + c;
          live[k][q] = act && a < ct.z.cnt && b < ct.y.cnt && c < ct.x.cnt;
          lid[k][q] = (a ? ct.z.t1 : ct.z.t0) + (b ? ct.y.t1 : ct.y.t0) +
                      (c ? ct.x.t1 : ct.x.t0);
          // a Dirichlet node's copies are not read
          x[k][q] = live[k][q] && !ct.masked ? v[lid[k][q]] : T(0);
        }
    box_advance(bx, step, pc);
  }
#pragma unroll
  for (int k = 0; k < GS_K; ++k) {
    const T acc = sum_copies(PER ? bx.order : 0, x[k]);
    if (masked[k]) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (live[k][q]) v[lid[k][q]] = T(0);
    } else if (cnt[k] == 1) {
      if (live[k][0] && !same_bits(acc, x[k][0])) v[lid[k][0]] = acc;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (live[k][q]) v[lid[k][q]] = acc;
    }
  }
}

static inline unsigned nblk(int64_t n, int t) {
  return (unsigned)((n + t - 1) / t);
}

template <class T, bool PER>
static void launch_gs_box(const sem_handle *h, T *v, hipStream_t s) {
  const Box bx = make_box(h->N, h->ex, h->ey, h->ez, h->dirichlet, h->periodic);
  const unsigned grid = nblk(h->nG, GS_T * GS_K);
  if (h->nL > (int64_t)UINT32_MAX)
    hipLaunchKernelGGL((k_gs_box<T, PER, true>), dim3(grid), dim3(GS_T), 0, s, bx, h->nG, v);
  else
    hipLaunchKernelGGL((k_gs_box<T, PER, false>), dim3(grid), dim3(GS_T), 0, s, bx, h->nG,
                       v);
}

template <class T> static void launch_gs_box_t(const sem_handle *h, T *v, hipStream_t s) {
  if (h->periodic != 0)
    launch_gs_box<T, true>(h, v, s);
  else
    launch_gs_box<T, false>(h, v, s);
}

void launch_gs(sem_handle *h, int prec, void *v, hipStream_t s) {
  if (h->nG == 0) return;
  if (prec == SEM_FP64)
    launch_gs_box_t<double>(h, (double *)v, s);
  else if (prec == SEM_FP32)
    launch_gs_box_t<float>(h, (float *)v, s);
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
