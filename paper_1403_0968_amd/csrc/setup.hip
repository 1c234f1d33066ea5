// Device-side setup: coordinates, geometric factors, lumped mass, Jacobi
// diagonal, reduced-precision copies.
//
// Geometry (paper section 4.2.1: chain rule and the G^T G metric,
// precomputed per elemental node; lumped mass J w_abc from discrete
// orthogonality).  Isoparametric: the derivatives X_r, X_s, X_t at a node are
// the derivative matrix applied to the mapped node positions along the three
// lines through it.  With the cofactor (cross-product) form
//   grad r = (X_s x X_t)/J,  grad s = (X_t x X_r)/J,  grad t = (X_r x X_s)/J,
//   J = X_r . (X_s x X_t),
// the weighted metric is G_ab = w_i w_j w_k kappa (c_a . c_b) / J with c_a the
// three cross products, and B = w_i w_j w_k J.  The mass term of equation
// semOperator, lumped by the quadrature, is H = alpha(X) B per local node;
// the Jacobi diagonal is that of the stiffness plus H.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "sem_internal.h"

namespace sem {

struct GeomParams {
  int N1, ex, ey, ez, mapping, M;
  double csig;  // sigma sqrt(2/M)
  double xi[17], w[17];
  double D[17 * 17];
};

__device__ inline void map_point(int mapping, double x, double y, double z,
                                 double &X, double &Y, double &Z) {
  const double tp = 2.0 * 3.14159265358979323846;
  X = x;
  Y = y;
  Z = z;
  if (mapping == SEM_MAP_SINE_X) {
    X = x + 0.05 * sin(tp * y) * sin(tp * z);
  } else if (mapping == SEM_MAP_SINE_CYCLIC) {
    const double sx = sin(tp * x), sy = sin(tp * y), sz = sin(tp * z);
    X = x + 0.05 * sy * sz;
    Y = y + 0.05 * sz * sx;
    Z = z + 0.05 * sx * sy;
  }
}

__global__ void k_geom(int64_t nL, GeomParams P, const double *__restrict__ omega,
                       const double *__restrict__ bph, double *__restrict__ X,
                       double *__restrict__ G, double *__restrict__ B,
                       double *__restrict__ kvert,
                       double *__restrict__ minJ_blk) {
  __shared__ double smin[256];
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double myJ = 1e300;
  if (l < nL) {
    const int N1 = P.N1, N3 = N1 * N1 * N1;
    const int64_t e = l / N3;
    const int p = (int)(l - e * N3);
    const int i = p % N1, j = (p / N1) % N1, k = p / (N1 * N1);
    const int64_t a = e % P.ex, b = (e / P.ex) % P.ey,
                  c = e / ((int64_t)P.ex * P.ey);
    const double hx = 1.0 / P.ex, hy = 1.0 / P.ey, hz = 1.0 / P.ez;
    auto ax_ = [&](int m) { return a * hx + (P.xi[m] + 1.0) * 0.5 * hx; };
    auto ay_ = [&](int m) { return b * hy + (P.xi[m] + 1.0) * 0.5 * hy; };
    auto az_ = [&](int m) { return c * hz + (P.xi[m] + 1.0) * 0.5 * hz; };
    double Xr[3] = {0, 0, 0}, Xs[3] = {0, 0, 0}, Xt[3] = {0, 0, 0};
    for (int m = 0; m < N1; ++m) {
      double q0, q1, q2;
      const double di = P.D[i * N1 + m], dj = P.D[j * N1 + m],
                   dk = P.D[k * N1 + m];
      map_point(P.mapping, ax_(m), ay_(j), az_(k), q0, q1, q2);
      Xr[0] += di * q0;
      Xr[1] += di * q1;
      Xr[2] += di * q2;
      map_point(P.mapping, ax_(i), ay_(m), az_(k), q0, q1, q2);
      Xs[0] += dj * q0;
      Xs[1] += dj * q1;
      Xs[2] += dj * q2;
      map_point(P.mapping, ax_(i), ay_(j), az_(m), q0, q1, q2);
      Xt[0] += dk * q0;
      Xt[1] += dk * q1;
      Xt[2] += dk * q2;
    }
    auto cross = [](const double *u, const double *v, double *o) {
      o[0] = u[1] * v[2] - u[2] * v[1];
      o[1] = u[2] * v[0] - u[0] * v[2];
      o[2] = u[0] * v[1] - u[1] * v[0];
    };
    double cr[3], cs[3], ct[3];
    cross(Xs, Xt, cr);
    cross(Xt, Xr, cs);
    cross(Xr, Xs, ct);
    const double J = Xr[0] * cr[0] + Xr[1] * cr[1] + Xr[2] * cr[2];
    double px, py, pz;
    map_point(P.mapping, ax_(i), ay_(j), az_(k), px, py, pz);
    X[l] = px;
    X[nL + l] = py;
    X[2 * nL + l] = pz;
    double kap = 1.0;
    if (P.M > 0) {
      double s = 0.0;
      for (int q = 0; q < P.M; ++q)
        s += cos(omega[3 * q] * px + omega[3 * q + 1] * py +
                 omega[3 * q + 2] * pz + bph[q]);
      kap = exp(P.csig * s);
    }
    // kappa at the element's 8 vertices, vertex v = a + 2 b + 4 c
    if ((i == 0 || i == N1 - 1) && (j == 0 || j == N1 - 1) &&
        (k == 0 || k == N1 - 1)) {
      const int v = (i ? 1 : 0) + (j ? 2 : 0) + (k ? 4 : 0);
      kvert[e * 8 + v] = kap;
    }
    const double wq = P.w[i] * P.w[j] * P.w[k];
    const double f = wq * kap / J;
    const double *cv[3] = {cr, cs, ct};
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    double *Ge = G + e * 6 * (int64_t)N3 + p;
    for (int q = 0; q < 6; ++q) {
      const double *u = cv[pa[q]], *v = cv[pb[q]];
      Ge[(int64_t)q * N3] = f * (u[0] * v[0] + u[1] * v[1] + u[2] * v[2]);
    }
    B[l] = wq * J;
    myJ = J;
  }
  smin[threadIdx.x] = myJ;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) minJ_blk[blockIdx.x] = smin[0];
}

// mass factor H = alpha(X) B (alpha_l from the nodal array, or the constant)
// with its FP32 and BF16 copies
__global__ void k_mass_factor(int64_t nL, double alpha,
                              const double *__restrict__ alpha_l,
                              const double *__restrict__ B, double *__restrict__ H,
                              float *__restrict__ H32, uint16_t *__restrict__ H16) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  const double a = alpha_l != nullptr ? alpha_l[l] : alpha;
  const double v = a * B[l];
  H[l] = v;
  H32[l] = (float)v;
  H16[l] = f32_to_bf16((float)v);
}

// unassembled diagonal of the local matrices (stiffness, plus H when the
// mesh has a mass term)
__global__ void k_diag(int64_t nL, int N1, const double *__restrict__ Dm,
                       const double *__restrict__ G, const double *__restrict__ H,
                       double *__restrict__ diag) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  const int N3 = N1 * N1 * N1;
  const int64_t e = l / N3;
  const int p = (int)(l - e * N3);
  const int i = p % N1, j = (p / N1) % N1, k = p / (N1 * N1);
  const double *Ge = G + e * 6 * (int64_t)N3;
  double s = 0.0;
  for (int m = 0; m < N1; ++m) {
    const double a = Dm[m * N1 + i], b = Dm[m * N1 + j], c = Dm[m * N1 + k];
    s += a * a * Ge[0 * N3 + m + N1 * j + N1 * N1 * k];
    s += b * b * Ge[3 * N3 + i + N1 * m + N1 * N1 * k];
    s += c * c * Ge[5 * N3 + i + N1 * j + N1 * N1 * m];
  }
  const double di = Dm[i * N1 + i], dj = Dm[j * N1 + j], dk = Dm[k * N1 + k];
  s += 2.0 * di * dj * Ge[1 * N3 + p] + 2.0 * di * dk * Ge[2 * N3 + p] +
       2.0 * dj * dk * Ge[4 * N3 + p];
  if (H != nullptr) s += H[l];
  diag[l] = s;
}

// inverse of the assembled diagonal (sum of copies in ascending local index)
__global__ void k_dinv(int64_t nG, const int32_t *__restrict__ off,
                       const int32_t *__restrict__ perm,
                       const uint8_t *__restrict__ gmask,
                       const double *__restrict__ diag, double *__restrict__ dinv,
                       float *__restrict__ dinv32) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nG) return;
  double s = 0.0;
  for (int q = off[g]; q < off[g + 1]; ++q) s = s + diag[perm[q]];
  const double v = gmask[g] ? 0.0 : 1.0 / s;
  dinv[g] = v;
  dinv32[g] = (float)v;
}

// reduced-precision copies; at n1 = 8 the BF16 copy is column-contiguous
// ([E][6][n1^2][n1], the layout the BF16 operator kernel reads)
__global__ void k_cast_geom(int64_t n, int N1, const double *__restrict__ G,
                            float *__restrict__ G32, uint16_t *__restrict__ G16) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float f = (float)G[q];
  G32[q] = f;
  int64_t d = q;
  if (N1 == 8) {
    const int64_t blk = q / 512;      // (element, factor)
    const int p = (int)(q - blk * 512);  // node i + 8 j + 64 k
    const int c = p % 64, k = p / 64;
    d = blk * 512 + c * 8 + k;
  }
  G16[d] = f32_to_bf16(f);
}

template <class T>
static void upload(DevBuf &b, const std::vector<T> &v, hipStream_t s) {
  b.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty())
    SEM_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T),
                           hipMemcpyHostToDevice, s));
}

void device_setup(sem_handle *h, const sem_mesh_desc *d, hipStream_t s) {
  const int T = 256;
  h->ref = make_ref_elem(d->N);
  HostMaps M = make_maps(d->N, d->ex, d->ey, d->ez, d->dirichlet, d->periodic);
  h->N = d->N;
  h->n1 = d->N + 1;
  h->ex = d->ex;
  h->ey = d->ey;
  h->ez = d->ez;
  h->dirichlet = d->dirichlet;
  h->periodic = d->periodic;
  h->mapping = d->mapping;
  h->has_mass = d->alpha_nodal != nullptr || d->alpha != 0.0;
  h->E = (int64_t)d->ex * d->ey * d->ez;
  h->nL = M.nL;
  h->nG = M.nG;

  upload(h->l2g, M.l2g, s);
  upload(h->perm, M.perm, s);
  upload(h->offsets, M.offsets, s);
  upload(h->mult, M.mult, s);
  upload(h->bmask, M.bmask, s);
  upload(h->gmask, M.gmask, s);
  upload(h->D64, h->ref.D, s);
  std::vector<float> D32(h->ref.D.begin(), h->ref.D.end());
  upload(h->D32, D32, s);
  // two-term BF16 split of D for the matrix-core operator
  std::vector<uint16_t> Dhi(D32.size()), Dlo(D32.size());
  for (size_t q = 0; q < D32.size(); ++q) {
    Dhi[q] = f32_to_bf16((float)h->ref.D[q]);
    Dlo[q] = f32_to_bf16((float)(h->ref.D[q] - (double)bf16_to_f32(Dhi[q])));
  }
  upload(h->D16hi, Dhi, s);
  upload(h->D16lo, Dlo, s);

  const int N1 = h->n1;
  GeomParams P{};
  P.N1 = N1;
  P.ex = d->ex;
  P.ey = d->ey;
  P.ez = d->ez;
  P.mapping = d->mapping;
  P.M = d->kappa_nfeat;
  P.csig = d->kappa_nfeat > 0 ? d->kappa_sigma * sqrt(2.0 / d->kappa_nfeat) : 0.0;
  for (int m = 0; m < N1; ++m) {
    P.xi[m] = h->ref.xi[m];
    P.w[m] = h->ref.w[m];
  }
  for (int q = 0; q < N1 * N1; ++q) P.D[q] = h->ref.D[q];

  DevBuf om, bp, minj;
  std::vector<double> omv, bv;
  if (d->kappa_nfeat > 0) {
    omv.assign(d->kappa_omega, d->kappa_omega + 3 * (size_t)d->kappa_nfeat);
    bv.assign(d->kappa_b, d->kappa_b + (size_t)d->kappa_nfeat);
  }
  upload(om, omv, s);
  upload(bp, bv, s);

  const int64_t nL = h->nL, nG = h->nG, nGeo = h->E * 6 * (int64_t)N1 * N1 * N1;
  h->coords.alloc(3 * nL * sizeof(double));
  h->G64.alloc(nGeo * sizeof(double));
  h->kvert.alloc(h->E * 8 * sizeof(double));
  h->G32.alloc(nGeo * sizeof(float));
  h->G16.alloc(nGeo * sizeof(uint16_t));
  h->mass.alloc(nL * sizeof(double));
  h->diag_L.alloc(nL * sizeof(double));
  h->dinv_G.alloc(nG * sizeof(double));
  h->dinv_G32.alloc(nG * sizeof(float));
  const unsigned gb = (unsigned)((nL + T - 1) / T);
  minj.alloc(gb * sizeof(double));
  hipLaunchKernelGGL(k_geom, dim3(gb), dim3(T), 0, s, nL, P, om.as<double>(),
                     bp.as<double>(), h->coords.as<double>(), h->G64.as<double>(),
                     h->mass.as<double>(), h->kvert.as<double>(),
                     minj.as<double>());
  SEM_HIP(hipGetLastError());
  DevBuf al;
  std::vector<double> av;  // lives until the stream is synchronised below
  if (h->has_mass) {
    if (d->alpha_nodal != nullptr) {
      av.assign(d->alpha_nodal, d->alpha_nodal + nL);
      for (double a : av)
        if (!(std::isfinite(a) && a >= 0.0))
          fail(SEM_ERR_ARG, "sem_setup: alpha_nodal values must be finite and >= 0");
      upload(al, av, s);
    }
    h->H64.alloc(nL * sizeof(double));
    h->H32.alloc(nL * sizeof(float));
    h->H16.alloc(nL * sizeof(uint16_t));
    hipLaunchKernelGGL(k_mass_factor, dim3(gb), dim3(T), 0, s, nL, d->alpha,
                       d->alpha_nodal != nullptr ? al.as<double>() : nullptr,
                       h->mass.as<double>(), h->H64.as<double>(),
                       h->H32.as<float>(), h->H16.as<uint16_t>());
    SEM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_diag, dim3(gb), dim3(T), 0, s, nL, N1, h->D64.as<double>(),
                     h->G64.as<double>(), h->has_mass ? h->H64.as<double>() : nullptr,
                     h->diag_L.as<double>());
  SEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dinv, dim3((unsigned)((nG + T - 1) / T)), dim3(T), 0, s,
                     nG, h->offsets.as<int32_t>(), h->perm.as<int32_t>(),
                     h->gmask.as<uint8_t>(), h->diag_L.as<double>(),
                     h->dinv_G.as<double>(), h->dinv_G32.as<float>());
  SEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_cast_geom, dim3((unsigned)((nGeo + T - 1) / T)), dim3(T),
                     0, s, nGeo, N1, h->G64.as<double>(), h->G32.as<float>(),
                     h->G16.as<uint16_t>());
  SEM_HIP(hipGetLastError());
  std::vector<double> mj(gb);
  SEM_HIP(hipMemcpyAsync(mj.data(), minj.p, gb * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  double mn = 1e300;
  for (double v : mj) mn = std::min(mn, v);
  if (!(mn > 0.0)) fail(SEM_ERR_ARG, "mapping is not invertible (J <= 0)");
}

}  // namespace sem
