// Host-side setup of libsem.so: the 1D reference element and the
// global-local maps of the structured hexahedral box.
//
// Reference element (paper section 4.2.1: Lagrange basis on the 1D
// Gauss-Lobatto-Legendre points):
//   nodes   -1, 1 and the zeros of P_N', found by Newton on P_N' with P_N''
//           taken from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P;
//   weights 2 / (N (N+1) P_N(x)^2);
//   D_im = l_m'(xi_i) from barycentric weights lambda_m = 1/prod(xi_m-xi_k):
//           D_im = (lambda_m/lambda_i)/(xi_i - xi_m), and D_ii = -sum_{m!=i} D_im
//           so that D applied to a constant is zero to roundoff.
//
// Maps (section 4.2.1, distinct global-local numbering after Fischer 1991):
// built directly from the lattice structure, without sorting.  A lattice
// coordinate t along a direction with E_d elements belongs to two elements
// when t is a multiple of N strictly inside (0, E_d N), else to one; the
// copies of a global node, visited with z outermost and the lower element
// first in every direction, come out in ascending local index.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "sem_internal.h"

namespace sem {

static void legendre_and_derivative(int N, double x, double &P, double &dP) {
  // P_{k+1} = ((2k+1) x P_k - k P_{k-1}) / (k+1);  P'_{k+1} = P'_{k-1} + (2k+1) P_k
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (N == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  P = p1;
  dP = d1;
}

RefElem make_ref_elem(int N) {
  if (N < 1 || N > 16) fail(SEM_ERR_ARG, "polynomial order N must be in 1..16");
  RefElem r;
  r.N = N;
  r.n1 = N + 1;
  r.xi.assign(r.n1, 0.0);
  r.w.assign(r.n1, 0.0);
  r.xi[0] = -1.0;
  r.xi[N] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i <= N / 2; ++i) {
    // search the i-th interior zero of P_N' in the left half; mirror it
    double x = -cos(pi * (i + 0.0) / N);
    for (int it = 0; it < 200; ++it) {
      double P, dP;
      legendre_and_derivative(N, x, P, dP);
      double d2P = (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x);
      double step = dP / d2P;
      x -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    if (2 * i == N) x = 0.0;
    r.xi[i] = x;
    r.xi[N - i] = -x;
  }
  for (int i = 0; i < r.n1; ++i) {
    double P, dP;
    legendre_and_derivative(N, r.xi[i], P, dP);
    r.w[i] = 2.0 / (N * (N + 1.0) * P * P);
  }
  std::vector<double> lam(r.n1, 1.0);
  for (int m = 0; m < r.n1; ++m) {
    double prod = 1.0;
    for (int k = 0; k < r.n1; ++k)
      if (k != m) prod *= (r.xi[m] - r.xi[k]);
    lam[m] = 1.0 / prod;
  }
  r.D.assign(r.n1 * r.n1, 0.0);
  for (int i = 0; i < r.n1; ++i) {
    double diag = 0.0;
    for (int m = 0; m < r.n1; ++m) {
      if (m == i) continue;
      double v = (lam[m] / lam[i]) / (r.xi[i] - r.xi[m]);
      r.D[i * r.n1 + m] = v;
      diag -= v;
    }
    r.D[i * r.n1 + i] = diag;
  }
  return r;
}

HostMaps make_maps(int N, int ex, int ey, int ez, int dirichlet, int periodic) {
  HostMaps M;
  const int n1 = N + 1;
  const int64_t n3 = (int64_t)n1 * n1 * n1;
  // a periodic direction (bit 1 x, 2 y, 4 z) identifies its faces at 0 and
  // 1: E_d N coordinates, the coordinate E_d N wrapping to 0
  const bool px = periodic & 1, py = periodic & 2, pz = periodic & 4;
  const int64_t Gx = (int64_t)ex * N + (px ? 0 : 1), Gy = (int64_t)ey * N + (py ? 0 : 1),
                Gz = (int64_t)ez * N + (pz ? 0 : 1);
  const int64_t E = (int64_t)ex * ey * ez;
  M.nL = E * n3;
  M.nG = Gx * Gy * Gz;
  if (M.nL >= (int64_t)INT32_MAX || M.nG >= (int64_t)INT32_MAX)
    fail(SEM_ERR_ARG, "mesh too large for 32-bit node indices");

  M.l2g.resize(M.nL);
  M.bmask.resize(M.nL);
  for (int64_t e = 0; e < E; ++e) {
    const int64_t a = e % ex, b = (e / ex) % ey, c = e / ((int64_t)ex * ey);
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const int64_t l = e * n3 + i + n1 * j + (int64_t)n1 * n1 * k;
          const int64_t gx = (a * N + i) % Gx, gy = (b * N + j) % Gy,
                        gz = (c * N + k) % Gz;
          M.l2g[l] = (int32_t)(gx + Gx * (gy + Gy * gz));
          const bool edge = (!px && (gx == 0 || gx == Gx - 1)) ||
                            (!py && (gy == 0 || gy == Gy - 1)) ||
                            (!pz && (gz == 0 || gz == Gz - 1));
          M.bmask[l] = (uint8_t)(dirichlet && edge);
        }
  }

  // per-direction owners of a lattice coordinate: (element, local index),
  // lower element first (coordinate 0 of a periodic direction: node 0 of
  // element 0 and node N of element Ed - 1)
  auto owners = [N](int64_t t, int64_t Ed, bool per, int64_t *el, int *loc) -> int {
    if (per && t == 0) {
      el[0] = 0;
      loc[0] = 0;
      el[1] = Ed - 1;
      loc[1] = N;
      return 2;
    }
    if (t % N == 0 && t > 0 && t < Ed * N) {
      el[0] = t / N - 1;
      loc[0] = N;
      el[1] = t / N;
      loc[1] = 0;
      return 2;
    }
    int64_t q = t / N;
    if (q >= Ed) q = Ed - 1;
    el[0] = q;
    loc[0] = (int)(t - q * N);
    return 1;
  };

  M.offsets.resize(M.nG + 1);
  M.perm.resize(M.nL);
  M.gmask.resize(M.nG);
  int64_t pos = 0;
  for (int64_t gz = 0; gz < Gz; ++gz) {
    int64_t elz[2], ely[2], elx[2];
    int lz[2], ly[2], lx[2];
    const int cz = owners(gz, ez, pz, elz, lz);
    for (int64_t gy = 0; gy < Gy; ++gy) {
      const int cy = owners(gy, ey, py, ely, ly);
      for (int64_t gx = 0; gx < Gx; ++gx) {
        const int cx = owners(gx, ex, px, elx, lx);
        const int64_t g = gx + Gx * (gy + Gy * gz);
        const bool onb = (!px && (gx == 0 || gx == Gx - 1)) ||
                         (!py && (gy == 0 || gy == Gy - 1)) ||
                         (!pz && (gz == 0 || gz == Gz - 1));
        const bool masked = dirichlet && onb;
        M.gmask[g] = (uint8_t)masked;
        M.offsets[g] = (int32_t)pos;
        const int64_t start = pos;
        for (int qz = 0; qz < cz; ++qz)
          for (int qy = 0; qy < cy; ++qy)
            for (int qx = 0; qx < cx; ++qx) {
              const int64_t e = elx[qx] + ex * (ely[qy] + (int64_t)ey * elz[qz]);
              const int64_t l = e * n3 + lx[qx] + n1 * ly[qy] +
                                (int64_t)n1 * n1 * lz[qz];
              M.perm[pos++] = (int32_t)l;
            }
        // ascending local index (a periodic direction with one element
        // puts its two copies in the same element, which the nesting above
        // does not order)
        std::sort(M.perm.begin() + start, M.perm.begin() + pos);
      }
    }
  }
  M.offsets[M.nG] = (int32_t)pos;
  if (pos != M.nL) fail(SEM_ERR_STATE, "internal: map construction lost nodes");
  M.mult.resize(M.nL);
  for (int64_t l = 0; l < M.nL; ++l) {
    const int32_t g = M.l2g[l];
    M.mult[l] = M.offsets[g + 1] - M.offsets[g];
  }
  return M;
}

}  // namespace sem
