// Reference-triangle operators of the nodal DG volume term (paper section
// 4.3.2; the nodal basis follows the nodal-DG textbook the paper cites):
//
//   nodes   warp-and-blend points (Warburton 2006): equidistant points of
//           the equilateral triangle displaced, along each edge direction,
//           by the blended interpolant of the shift from equidistant to
//           Gauss-Lobatto points, then mapped to the reference triangle
//           (vertices (-1,-1), (1,-1), (-1,1)); order: rows n = 0..N from
//           the edge s = -1, m = 0..N-n along a row;
//   basis   orthonormal psi_ij = sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i in
//           collapsed coordinates a = 2(1+r)/(1-s) - 1, b = s;
//   V       V_nk = psi_k(node n); Dr = Vr V^-1, Ds = Vs V^-1;
//   mass    M = (V V^T)^-1 = V^-T V^-1;
//   weak    Drw = M^-1 Dr^T M, Dsw = M^-1 Ds^T M (the volume integrals
//           <F, dv/dr> against every basis function, after M^-1).
#include <cmath>
#include <vector>

#include "sem_internal.h"

namespace sem {

// optimised blending parameter per order (textbook table, N = 1..15)
static const double kAlphaOpt[15] = {0.0000, 0.0000, 1.4152, 0.1001, 0.2751,
                                     0.9800, 1.0999, 1.2832, 1.3648, 1.4773,
                                     1.4959, 1.5743, 1.5770, 1.6223, 1.6258};

// Jacobi polynomial P_n^(a,b)(x), classical normalisation, three-term
// recurrence in n
static double jacobi(double x, double a, double b, int n) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k + a + b;
    const double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
    const double a2 = (c - 1.0) * (a * a - b * b);
    const double a3 = (c - 2.0) * (c - 1.0) * c;
    const double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// squared norm of P_n^(a,b) under the weight (1-x)^a (1+x)^b on [-1, 1]
static double jacobi_norm2(double a, double b, int n) {
  return std::pow(2.0, a + b + 1.0) / (2.0 * n + a + b + 1.0) *
         std::tgamma(n + a + 1.0) * std::tgamma(n + b + 1.0) /
         (std::tgamma(n + a + b + 1.0) * std::tgamma(n + 1.0));
}

// orthonormal P_n and its derivative (d/dx P_n^(a,b) = (n+a+b+1)/2
// P_{n-1}^(a+1,b+1))
static double pn(double x, double a, double b, int n) {
  return jacobi(x, a, b, n) / std::sqrt(jacobi_norm2(a, b, n));
}
static double dpn(double x, double a, double b, int n) {
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi(x, a + 1.0, b + 1.0, n - 1) /
         std::sqrt(jacobi_norm2(a, b, n));
}

static double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// psi_ij and its r- and s-derivatives at (r, s)
static void basis_and_gradient(double r, double s, int i, int j, double &f,
                               double &fr, double &fs) {
  const double b = s;
  const double a = (std::fabs(s - 1.0) > 1e-13) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  const double pa = pn(a, 0.0, 0.0, i), dpa = dpn(a, 0.0, 0.0, i);
  const double pb = pn(b, 2.0 * i + 1.0, 0.0, j), dpb = dpn(b, 2.0 * i + 1.0, 0.0, j);
  const double rt2 = std::sqrt(2.0);
  f = rt2 * pa * pb * ipow(1.0 - b, i);
  // d/dr: da/dr = 2 / (1 - b);  d/ds: da/ds = (1 + a) / (1 - b)
  fr = i > 0 ? rt2 * 2.0 * dpa * pb * ipow(1.0 - b, i - 1) : 0.0;
  fs = rt2 * pa * (dpb * ipow(1.0 - b, i) - (i > 0 ? i * pb * ipow(1.0 - b, i - 1) : 0.0));
  if (i > 0) fs += rt2 * dpa * (1.0 + a) * pb * ipow(1.0 - b, i - 1);
}

// warp function: barycentric interpolant on the N+1 equidistant points of
// the shift to the Gauss-Lobatto points, divided by (1 - x^2) inside
static double warp(int N, const std::vector<double> &gl, double x) {
  std::vector<double> xe(N + 1), wb(N + 1);
  double binom = 1.0;
  for (int i = 0; i <= N; ++i) {
    xe[i] = -1.0 + 2.0 * i / N;
    wb[i] = (i % 2 ? -1.0 : 1.0) * binom;  // barycentric weights (equidistant)
    binom = binom * (N - i) / (i + 1.0);
  }
  double num = 0.0, den = 0.0, w = 0.0;
  bool exact = false;
  for (int i = 0; i <= N; ++i) {
    const double d = x - xe[i];
    if (std::fabs(d) < 1e-15) {
      w = gl[i] - xe[i];
      exact = true;
      break;
    }
    num += wb[i] / d * (gl[i] - xe[i]);
    den += wb[i] / d;
  }
  if (!exact) w = num / den;
  if (std::fabs(x) < 1.0 - 1e-10) w /= (1.0 - x * x);
  return w;
}

static void gauss_jordan_inverse(std::vector<double> &A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(A[i * n + c]) > std::fabs(A[p * n + c])) p = i;
    if (A[p * n + c] == 0.0) fail(SEM_ERR_ARG, "dg: singular Vandermonde matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[p * n + k]);
      std::swap(I[c * n + k], I[p * n + k]);
    }
    const double inv = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= inv;
      I[c * n + k] *= inv;
    }
    for (int i = 0; i < n; ++i) {
      if (i == c) continue;
      const double f = A[i * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[i * n + k] -= f * A[c * n + k];
        I[i * n + k] -= f * I[c * n + k];
      }
    }
  }
  A.swap(I);
}

static std::vector<double> matmul(const std::vector<double> &A,
                                  const std::vector<double> &B, int n,
                                  bool transA = false, bool transB = false) {
  std::vector<double> C(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double a = transA ? A[k * n + i] : A[i * n + k];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[i * n + j] += a * (transB ? B[j * n + k] : B[k * n + j]);
    }
  return C;
}

DgRef make_dg_ref(int N) {
  if (N < 1 || N > 8) fail(SEM_ERR_ARG, "dg: N must be in 1..8");
  DgRef R;
  R.N = N;
  R.Np = (N + 1) * (N + 2) / 2;
  const int Np = R.Np;
  const std::vector<double> gl = make_ref_elem(N).xi;  // Gauss-Lobatto points
  const double alpha = kAlphaOpt[N - 1];
  const double s3 = std::sqrt(3.0), pi = 3.14159265358979323846;
  for (int n = 0; n <= N; ++n)
    for (int m = 0; m <= N - n; ++m) {
      const double L1 = (double)n / N, L3 = (double)m / N, L2 = 1.0 - L1 - L3;
      double x = -L2 + L3, y = (-L2 - L3 + 2.0 * L1) / s3;
      const double w1 = 4.0 * L2 * L3 * warp(N, gl, L3 - L2) * (1.0 + (alpha * L1) * (alpha * L1));
      const double w2 = 4.0 * L1 * L3 * warp(N, gl, L1 - L3) * (1.0 + (alpha * L2) * (alpha * L2));
      const double w3 = 4.0 * L1 * L2 * warp(N, gl, L2 - L1) * (1.0 + (alpha * L3) * (alpha * L3));
      x += w1 + std::cos(2.0 * pi / 3.0) * w2 + std::cos(4.0 * pi / 3.0) * w3;
      y += std::sin(2.0 * pi / 3.0) * w2 + std::sin(4.0 * pi / 3.0) * w3;
      const double l1 = (s3 * y + 1.0) / 3.0;
      const double l2 = (-3.0 * x - s3 * y + 2.0) / 6.0;
      const double l3 = (3.0 * x - s3 * y + 2.0) / 6.0;
      R.r.push_back(-l2 + l3 - l1);
      R.s.push_back(-l2 - l3 + l1);
    }
  std::vector<double> V(Np * Np), Vr(Np * Np), Vs(Np * Np);
  for (int n = 0; n < Np; ++n) {
    int k = 0;
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j <= N - i; ++j, ++k)
        basis_and_gradient(R.r[n], R.s[n], i, j, V[n * Np + k], Vr[n * Np + k],
                           Vs[n * Np + k]);
  }
  std::vector<double> Vinv = V;
  gauss_jordan_inverse(Vinv, Np);
  R.Dr = matmul(Vr, Vinv, Np);
  R.Ds = matmul(Vs, Vinv, Np);
  const std::vector<double> M = matmul(Vinv, Vinv, Np, true, false);    // V^-T V^-1
  const std::vector<double> Minv = matmul(V, V, Np, false, true);       // V V^T
  R.Drw = matmul(matmul(Minv, R.Dr, Np, false, true), M, Np);           // M^-1 Dr^T M
  R.Dsw = matmul(matmul(Minv, R.Ds, Np, false, true), M, Np);
  return R;
}

}  // namespace sem
