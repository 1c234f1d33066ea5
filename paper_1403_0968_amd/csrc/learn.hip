// Learned per-element coarse correction on a mesh (the preconditioner slot
// that section 4.2.2 leaves open): the element coarse operators that the
// network predicts from the element's kappa, their application inside
// flexible CG, and the generation of training pairs from FP64 solves
// followed by GPU training.
//
// Coarse space: bubble basis b_a(x) = (1 - x^2) P_a(x), a = 0..p,
// p = min(2, N-2), B = tensor products on the interior nodes (K = (p+1)^3
// columns), every column scaled so that the reference element's coarse
// inverse has unit diagonal.  The exact element coarse correction is
// B G_e^{-1} B^T r_I with G_e = B^T A_II B (A_II the element stiffness on
// its interior nodes).  The network (n_in = 8, n_out = K(K+1)/2) maps the 8
// log-kappa vertex deviations of an element to a lower-triangular L with
// M_e = L L^T ~ kappa_e h_e G_e^{-1}, and the correction
//   c_I = damping B (M_e / (kappa_e h_e)) B^T r_I
// is symmetric positive semi-definite whatever the network outputs
// (kappa_e: mean of the vertex values, h_e: element size).  The exact
// operators themselves (no network) can be attached instead, which gives
// the correction the network is trained to imitate.
// Training pairs: y = B^T r_I / ||B^T r_I|| from a snapshot residual of an
// FP64 Jacobi-PCG solve (or, for a random half of the pairs, a random unit
// direction) with target alpha* = kappa_e h_e G_e^{-1} y; the loss is the
// mean of (L L^T y - alpha*)^2.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <random>
#include <vector>

#include "ax_tile.h"

namespace sem {

struct CoarseTab {
  float B1[7][3];  // B1[i][a] = (1 - x_i^2) P_a(x_i) at interior GLL point i
  float sc[27];    // column scale of B, column a + Q (b + Q c)
};

// Per-mesh state: basis B [ni][K] (FP64; its FP32 factors B1 and column
// scale sc for the apply kernel, sc also on the device), kappa features of
// every element (FP32 [E][8] and BF16 network input rows [E][ldx]), the
// element operators M_e / (kappa_e h_e) (FP32, symmetric, packed lower
// triangles [E][K(K+1)/2], row a holding columns 0..a) of the network of
// version mver or of the exact inverses, and the corrections (unique-node
// vector cG for the solver, E-vector cL for sem_precond_apply).
struct Learn {
  int K = 0, ni = 0, ldx = 16, ldo = 16;
  DevBuf Bd, Xk, Ml, cG, cL, Sc, O, kfeat, invkh;
  DevBuf ep;  // flexible CG: element terms of (r, c) and (c, w), [2][E]
  CoarseTab tab{};
  const sem_mlp *mnet = nullptr;
  uint64_t mver = 0;
  bool exact = false;          // Ml holds the exact inverses (no network)
  double exact_damping = 0.0;  // damping of the exact correction
  DevBuf exact_damp_dev;       // its device copy (float)
};

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

// ---------------------------------------------------------------------------
// coarse layout kernels
// ---------------------------------------------------------------------------
// interior index q of local node (i, j, k), or -1 on the element's faces
__device__ inline int interior_index(int i, int j, int k, int n1) {
  const int N = n1 - 1, m = N - 1;
  if (i < 1 || i >= N || j < 1 || j >= N || k < 1 || k >= N) return -1;
  return (i - 1) + m * ((j - 1) + m * (k - 1));
}

// Exact normalised coarse inverses, one workgroup per element: for every
// bubble column b_k the element operator (shared element routine, FP64,
// zero face values) gives A_II b_k through the element's scratch rows U, W;
// column k of G_e = B^T A_II B is reduced over the workgroup; thread 0 then
// inverts the symmetrised G_e by Cholesky and stores kappa_e h_e G_e^{-1}.
// A G_e that is not positive definite is stored as NaN.
template <int N1, int NT>
__global__ void __launch_bounds__(NT)
    k_coarse_exact(int64_t E, const double *__restrict__ G,
                   const double *__restrict__ D, const double *__restrict__ Bd,
                   int K, double *__restrict__ U, double *__restrict__ W,
                   const double *__restrict__ kv, double hsz,
                   double *__restrict__ Mex) {
  constexpr int NP = N1 * N1, N3 = NP * N1, N = N1 - 1;
  __shared__ double smem[lds_words<N1>(1)];
  __shared__ double red[NT / 64];
  __shared__ double Gs[27 * 27];
  const int64_t e = blockIdx.x;
  if (e >= E) return;  // uniform
  const int t = threadIdx.x;
  const bool act = t < NP;
  const int c = act ? t : 0;
  const int i = c % N1, j = c / N1;
  double *u = U + e * N3, *w = W + e * N3;
  for (int kb = 0; kb < K; ++kb) {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const int q = act ? interior_index(i, j, k, N1) : -1;
      if (act) u[c + k * NP] = q >= 0 ? Bd[q * K + kb] : 0.0;
    }
    ax_tile<N1, 1, double, double, double, double, false, false>(
        t, 0, 1, D, G + e * 6 * N3, u, w, nullptr, smem);
    double wc[N1];
    int qc[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      qc[k] = act ? interior_index(i, j, k, N1) : -1;
      wc[k] = qc[k] >= 0 ? w[c + k * NP] : 0.0;  // this thread's own column
    }
    for (int jb = 0; jb < K; ++jb) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < N1; ++k)
        if (qc[k] >= 0) a += Bd[qc[k] * K + jb] * wc[k];
      a = block_allsum<NT>(a, red);
      if (t == 0) Gs[jb * K + kb] = a;
    }
  }
  __syncthreads();
  if (t != 0) return;  // no barrier follows
  (void)N;
  // Cholesky of the symmetrised G_e in the lower triangle of Gs
  bool ok = true;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < a; ++b) {
      const double v = 0.5 * (Gs[a * K + b] + Gs[b * K + a]);
      Gs[a * K + b] = v;
      Gs[b * K + a] = v;
    }
  for (int jj = 0; jj < K && ok; ++jj) {
    double d = Gs[jj * K + jj];
    for (int k = 0; k < jj; ++k) d -= Gs[jj * K + k] * Gs[jj * K + k];
    if (!(d > 0.0)) {
      ok = false;
      break;
    }
    const double ljj = sqrt(d);
    Gs[jj * K + jj] = ljj;
    for (int ii = jj + 1; ii < K; ++ii) {
      double v = Gs[ii * K + jj];
      for (int k = 0; k < jj; ++k) v -= Gs[ii * K + k] * Gs[jj * K + k];
      Gs[ii * K + jj] = v / ljj;
    }
  }
  double kbar = 0.0;
  for (int v = 0; v < 8; ++v) kbar += kv[e * 8 + v] / 8.0;
  const double scale = kbar * hsz;  // kappa_e h_e
  double *Me = Mex + e * K * K;
  for (int col = 0; col < K; ++col) {
    double y[27];
    for (int ii = 0; ii < K; ++ii) {  // L y = e_col
      double v = ii == col ? 1.0 : 0.0;
      for (int k = 0; k < ii; ++k) v -= Gs[ii * K + k] * y[k];
      y[ii] = v / Gs[ii * K + ii];
    }
    for (int ii = K - 1; ii >= 0; --ii) {  // L^T x = y
      double v = y[ii];
      for (int k = ii + 1; k < K; ++k) v -= Gs[k * K + ii] * y[k];
      y[ii] = v / Gs[ii * K + ii];
    }
    for (int ii = 0; ii < K; ++ii) Me[ii * K + col] = ok ? y[ii] * scale : NAN;
  }
}

// coarse training pairs, one 64-thread workgroup per pair: y = B^T r_I /
// ||B^T r_I|| from the snapshot residual or, where piso[p] is set, the
// caller's random unit vector yr[p] (so that every direction of the K x K
// operator is constrained, not only those the residuals excite);
// alpha* = Mex_e y; T[p] = [y, alpha*] (FP32), X[p] = the element's kappa
// features (BF16, zero padding)
__global__ void __launch_bounds__(64)
    k_coarse_pairs(int np, const int32_t *__restrict__ psnap,
                   const int32_t *__restrict__ pelem, int64_t nG, int n1,
                   const int32_t *__restrict__ l2g, const double *__restrict__ rs,
                   const double *__restrict__ Bd, int K, int ni,
                   const double *__restrict__ Mex, const float *__restrict__ kf,
                   const int32_t *__restrict__ piso, const double *__restrict__ yr,
                   uint16_t *__restrict__ X, int ldx, float *__restrict__ T) {
  __shared__ double rI[343];
  __shared__ double y[27];
  const int p = blockIdx.x;
  if (p >= np) return;
  const int t = threadIdx.x;
  const int n3 = n1 * n1 * n1, m = n1 - 2;
  const int64_t e = pelem[p];
  const double *r = rs + (int64_t)psnap[p] * nG;
  const bool iso = piso[p] != 0;  // uniform per block
  if (!iso)
    for (int q = t; q < ni; q += 64) {
      const int i = q % m + 1, j = (q / m) % m + 1, k = q / (m * m) + 1;
      rI[q] = r[l2g[e * n3 + i + n1 * (j + n1 * k)]];
    }
  __syncthreads();
  double yj = 0.0;
  if (t < K) {
    if (iso)
      yj = yr[(size_t)p * K + t];
    else
      for (int q = 0; q < ni; ++q) yj += Bd[q * K + t] * rI[q];
  }
  const double nrm = sqrt(wave_sum(yj * yj));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  if (t < K) y[t] = yj * inv;
  __syncthreads();
  float *tp = T + (size_t)p * 2 * K;
  if (t < K) {
    double a = 0.0;
    for (int jj = 0; jj < K; ++jj) a += Mex[(e * K + t) * K + jj] * y[jj];
    tp[t] = (float)y[t];
    tp[K + t] = (float)a;
  }
  uint16_t *xp = X + (size_t)p * ldx;
  for (int q = t; q < ldx; q += 64)
    xp[q] = q < 8 ? f32_to_bf16(kf[e * 8 + q]) : (uint16_t)0;
}

// element operators from the network outputs: M_e = invkh_e L L^T, packed
// lower triangle (entry (a, b) and (b, a) are the same sum of the same
// products, so one copy loses nothing)
__global__ void __launch_bounds__(256)
    k_factor_to_M(int64_t E, int K, const float *__restrict__ O, int ldo,
                  const float *__restrict__ invkh, float *__restrict__ Ml) {
  const int64_t e = blockIdx.x;
  const float *o = O + e * ldo;
  const float sc = invkh[e];
  const int kp = K * (K + 1) / 2;
  for (int ab = threadIdx.x; ab < kp; ab += 256) {  // packed row a, column b <= a
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= ab) ++a;
    const int b = ab - a * (a + 1) / 2;
    float v = 0.f;
    for (int c = 0; c <= b; ++c) v += o[a * (a + 1) / 2 + c] * o[b * (b + 1) / 2 + c];
    Ml[e * kp + ab] = sc * v;
  }
}

// element operators from exact inverses: M_e / (kappa_e h_e) with
// M_e = kappa_e h_e G_e^{-1} (Mex, FP64 [E][K][K], symmetrised), packed
// lower triangle in FP32
__global__ void __launch_bounds__(256)
    k_exact_to_M(int64_t E, int K, const double *__restrict__ Mex,
                 const float *__restrict__ invkh, float *__restrict__ Ml) {
  const int64_t e = blockIdx.x;
  const double *M = Mex + e * K * K;
  const double sc = (double)invkh[e];
  const int kp = K * (K + 1) / 2;
  for (int ab = threadIdx.x; ab < kp; ab += 256) {
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= ab) ++a;
    const int b = ab - a * (a + 1) / 2;
    Ml[e * kp + ab] = (float)(sc * 0.5 * (M[a * K + b] + M[b * K + a]));
  }
}

// correction of the coarse layout: c = damping B M_e B^T r_I on the interior
// nodes of every element.  UNIQUE: r on unique nodes (read through the box
// numbering) and c written to the interior entries of the unique-node
// vector out (its other entries stay zero); otherwise r is a continuous
// E-vector and out the E-vector of element corrections, zero on the faces.
// The basis is a tensor product with a column scale, B = (B1 x B1 x B1)
// diag(sc) (B1: the Q 1D bubbles on the M interior points), so both
// products are sum-factorised: y = sc o (B1^T x B1^T x B1^T) r_I in three
// contractions of one direction each, then alpha = damping M_e y, then
// c = (B1 x B1 x B1)(sc o alpha) in three more (M = 6, Q = 3: 1.1 k instead
// of 5.8 k multiply-adds each way).  One wave per element, persistent, no workgroup barrier: lane
// p < M^2 owns the pencil (j, k) of M contiguous interior nodes, the
// intermediate tensors pass through the wave's LDS region, and the loads of
// the wave's next element (its pencil values and M_e, a packed triangle of
// K(K+1)/2 words) are issued before the current element's contractions.  (The dense form, one wave per element
// with B in LDS: 43 us per apply at 24^3 elements, N = 7, bound by its LDS
// and vector instruction count.)
constexpr int CA_WAVES = 4;


// FUSE (with UNIQUE): the flexible-CG iteration's preconditioner step.  zf
// is the search vector z of the solve, holding dinv o r on entry; the
// correction is added to it in place (z = dinv o r + c, as the separate
// correction-then-sum order gives: c is rounded to FP32 first), and every
// element stores its terms of the two dot products that involve c,
// epart[e] = (r_I, c) and epart[E + e] = (c, w_I), with w_I the element's
// interior values of the operator output wL (single copies: the assembled
// values), summed by a fixed butterfly over the wave.
template <class TV, bool UNIQUE, int M, int Q, bool FUSE = false>
__global__ void __launch_bounds__(64 * CA_WAVES)
    k_coarse_apply(int64_t E, Box box, CoarseTab tb, const float *__restrict__ scg,
                   const TV *__restrict__ r, const float *__restrict__ Ml,
                   const float *__restrict__ damping, float *__restrict__ out,
                   TV *__restrict__ zf = nullptr, const TV *__restrict__ wL = nullptr,
                   double *__restrict__ epart = nullptr) {
  static_assert(!FUSE || UNIQUE, "the fused step works on unique-node vectors");
  constexpr int K = Q * Q * Q, KK = K * (K + 1) / 2, MR = (KK + 63) / 64, P = M * M;
  constexpr int N1 = M + 2, N3 = N1 * N1 * N1, Q2 = Q * Q;
  constexpr int REG = Q * P + Q2 * M + 2 * 32 + KK;  // floats per wave
  __shared__ float ca_lds[CA_WAVES * REG];
  const int wave = threadIdx.x >> 6, t = threadIdx.x & 63;
  float *s1 = ca_lds + wave * REG;  // [Q][P]  (a, pencil)
  float *s2 = s1 + Q * P;           // [M][Q2] (k, a + Q b)
  float *yv = s2 + Q2 * M;          // [K]
  float *bv = yv + 32;              // [K]
  float *Ms = bv + 32;              // M_e, packed lower triangle
  const float damp = damping[0];
  const float sct = t < K ? scg[t] : 0.f;
  // first interior node of this lane's pencil (j, k) = (t % M, t / M)
  const int pj = t % M + 1, pk = min(t / M, M - 1) + 1;
  const int64_t offp = UNIQUE ? 1 + (int64_t)box.Gx * pj + box.Gxy * pk
                              : 1 + (int64_t)N1 * (pj + N1 * pk);
  auto base = [&](int64_t e) -> int64_t {
    return UNIQUE ? box_origin(box, (uint32_t)e) : e * N3;
  };
  const int64_t stride = (int64_t)gridDim.x * CA_WAVES;
  int64_t e = (int64_t)blockIdx.x * CA_WAVES + wave;
  TV rv[M];
  float mv[MR];
  auto fetch = [&](int64_t en) {
    const int64_t g = base(en) + offp;
#pragma unroll
    for (int i = 0; i < M; ++i) rv[i] = t < P ? r[g + i] : TV(0);
    const float *Me = Ml + en * KK;
#pragma unroll
    for (int i = 0; i < MR; ++i) mv[i] = t + 64 * i < KK ? Me[t + 64 * i] : 0.f;
  };
  if (e < E) fetch(e);
  for (; e < E; e += stride) {
    TV rcur[FUSE ? M : 1];  // this element's r (rv is refilled by the prefetch)
    if constexpr (FUSE) {
#pragma unroll
      for (int i = 0; i < M; ++i) rcur[i] = rv[i];
    }
    // restriction, direction i (registers): s1[a][pencil]
    if (t < P) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < M; ++i) acc += tb.B1[i][a] * (float)rv[i];
        s1[a * P + t] = acc;
      }
    }
#pragma unroll
    for (int i = 0; i < MR; ++i)
      if (t + 64 * i < KK) Ms[t + 64 * i] = mv[i];
    wave_lds_sync();
    // FUSE: this element's z and w_I are read now, so that their latency
    // overlaps the contractions below (with one element per wave the
    // prefetch of the next element's r and M_e does not apply)
    TV zv[FUSE ? M : 1], wv[FUSE ? M : 1];
    if constexpr (FUSE) {
      if (t < P) {
        const int64_t g = base(e) + offp;
        const int64_t l = e * N3 + 1 + (int64_t)N1 * (pj + N1 * pk);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          zv[i] = zf[g + i];
          wv[i] = wL[l + i];
        }
      }
    }
    if (e + stride < E) fetch(e + stride);
    // direction j: lane (a, k) -> s2[k][a + Q b]
    if (t < Q * M) {
      const int a = t % Q, k = t / Q;
      float v[M];
#pragma unroll
      for (int j = 0; j < M; ++j) v[j] = s1[a * P + j + M * k];
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < M; ++j) acc += tb.B1[j][b] * v[j];
        s2[k * Q2 + a + Q * b] = acc;
      }
    }
    wave_lds_sync();
    // direction k: lane ab -> y[ab + Q2 c] (unscaled)
    if (t < Q2) {
      float v[M];
#pragma unroll
      for (int k = 0; k < M; ++k) v[k] = s2[k * Q2 + t];
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < M; ++k) acc += tb.B1[k][c] * v[k];
        yv[t + Q2 * c] = acc;
      }
    }
    wave_lds_sync();
    // alpha = damping M_e (sc o y); beta = sc o alpha
    if (t < K) {
      float acc = 0.f;
#pragma unroll
      for (int jj = 0; jj < K; ++jj)  // M_e[jj][t] (M_e is symmetric)
        acc += Ms[jj >= t ? jj * (jj + 1) / 2 + t : t * (t + 1) / 2 + jj] *
               (tb.sc[jj] * yv[jj]);
      bv[t] = sct * (damp * acc);
    }
    wave_lds_sync();
    // prolongation, direction k: lane ab -> s2[k][ab]
    if (t < Q2) {
      float v[Q];
#pragma unroll
      for (int c = 0; c < Q; ++c) v[c] = bv[t + Q2 * c];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        float acc = 0.f;
#pragma unroll
        for (int c = 0; c < Q; ++c) acc += tb.B1[k][c] * v[c];
        s2[k * Q2 + t] = acc;
      }
    }
    wave_lds_sync();
    // direction j: lane (a, k) -> s1[a][j + M k]
    if (t < Q * M) {
      const int a = t % Q, k = t / Q;
      float v[Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) v[b] = s2[k * Q2 + a + Q * b];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int b = 0; b < Q; ++b) acc += tb.B1[j][b] * v[b];
        s1[a * P + j + M * k] = acc;
      }
    }
    wave_lds_sync();
    // direction i: lane = pencil, M contiguous interior nodes
    double prc = 0.0, pcw = 0.0;  // FUSE: this lane's (r_I, c), (c, w_I) terms
    if (t < P) {
      float v[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) v[a] = s1[a * P + t];
      const int64_t g = base(e) + offp;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < Q; ++a) acc += tb.B1[i][a] * v[a];
        if constexpr (FUSE) {
          const TV c = (TV)acc;
          zf[g + i] = zv[i] + c;
          prc += (double)rcur[i] * (double)c;
          pcw += (double)c * (double)wv[i];
        } else {
          out[g + i] = acc;
        }
      }
    }
    if constexpr (FUSE) {
      prc = wave_sum(prc);
      pcw = wave_sum(pcw);
      if (t == 0) {
        epart[e] = prc;
        epart[E + e] = pcw;
      }
    }
    if (!UNIQUE)  // the faces of the element carry no correction
      for (int p = t; p < N3; p += 64) {
        const int i = p % N1, j = (p / N1) % N1, k = p / (N1 * N1);
        if (interior_index(i, j, k, N1) < 0) out[e * N3 + p] = 0.f;
      }
    wave_lds_sync();  // the LDS region is rewritten for the next element
  }
}

// device damping of the attached correction (network or exact operators)
static const float *learn_damping_dev(const sem_handle *h) {
  return h->learn->exact ? h->learn->exact_damp_dev.as<float>()
                         : mlp_damping_dev(h->net);
}

template <class TV, bool UNIQUE, int M, int Q, bool FUSE>
static void launch_ca(const sem_handle *h, const Learn *L, const TV *r, float *out,
                      TV *zf, const TV *wL, double *epart, hipStream_t s) {
  const Box box = UNIQUE ? make_box(h->N, h->ex, h->ey, h->ez, h->dirichlet, h->periodic) : Box{};
  const int64_t groups = (h->E + CA_WAVES - 1) / CA_WAVES;
  const unsigned grid = (unsigned)groups;
  hipLaunchKernelGGL((k_coarse_apply<TV, UNIQUE, M, Q, FUSE>), dim3(grid),
                     dim3(64 * CA_WAVES), 0, s, h->E, box, L->tab, L->Sc.as<float>(), r,
                     L->Ml.as<float>(), learn_damping_dev(h), out, zf, wL, epart);
}

template <class TV, bool UNIQUE, bool FUSE = false>
static void launch_coarse_apply(const sem_handle *h, const Learn *L, const TV *r,
                                float *out, hipStream_t s, TV *zf = nullptr,
                                const TV *wL = nullptr, double *epart = nullptr) {
  switch (h->N) {
#define SEM_CA(NN, MM, QQ)                                                      \
  case NN:                                                                      \
    launch_ca<TV, UNIQUE, MM, QQ, FUSE>(h, L, r, out, zf, wL, epart, s);       \
    break;
    SEM_CA(2, 1, 1)
    SEM_CA(3, 2, 2)
    SEM_CA(4, 3, 3)
    SEM_CA(5, 4, 3)
    SEM_CA(6, 5, 3)
    SEM_CA(7, 6, 3)
    SEM_CA(8, 7, 3)
#undef SEM_CA
    default: fail(SEM_ERR_STATE, "coarse layout: N must be in 2..8");
  }
  SEM_HIP(hipGetLastError());
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

// a network fits the coarse layout of this mesh when n_in = 8 and
// n_out = K(K+1)/2 (N >= 2); the element targets are those of the stiffness
// operator alone (no mass term)
static int coarse_k(const sem_handle *h) {
  const int q = std::min(2, h->N - 2) + 1;
  return q * q * q;
}

static void check_mesh(const sem_handle *h) {
  if (h->N < 2 || h->N > 8)
    fail(SEM_ERR_ARG, "learned correction: N must be in 2..8");
  if (h->has_mass)
    fail(SEM_ERR_STATE, "learned correction: meshes with a mass term "
                        "(alpha != 0) are not supported");
}

static void check_net(const sem_handle *h, const sem_mlp *net) {
  check_mesh(h);
  int n_in = 0, n_out = 0;
  mlp_info(net, &n_in, nullptr, &n_out, nullptr, nullptr);
  const int K = coarse_k(h);
  if (n_in != 8 || n_out != K * (K + 1) / 2)
    fail(SEM_ERR_ARG, "learned correction: the network needs n_in = 8 and "
                      "n_out = K(K+1)/2 with K = (min(2, N-2)+1)^3");
}

// inverse of a small dense matrix (Gauss-Jordan with partial pivoting, FP64)
static std::vector<double> small_inverse(std::vector<double> A, int n) {
  std::vector<double> X((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) X[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
    if (!(std::fabs(A[(size_t)piv * n + c]) > 0.0))
      fail(SEM_ERR_STATE, "coarse layout: singular reference coarse matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
      std::swap(X[(size_t)c * n + k], X[(size_t)piv * n + k]);
    }
    const double d = A[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      A[(size_t)c * n + k] /= d;
      X[(size_t)c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * n + c];
      for (int k = 0; k < n; ++k) {
        A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
        X[(size_t)r * n + k] -= f * X[(size_t)c * n + k];
      }
    }
  }
  return X;
}

// bubble basis on the host (FP64): B[q][col], q = interior node (i fastest),
// col = a + q1 b + q1^2 c, b_a(x) = (1 - x^2) P_a(x), a <= 2, every column
// scaled by sqrt of the matching diagonal entry of the reference coarse
// inverse.  Reference: the unit cube with kappa = 1 (kappa h = 1), whose
// stiffness is (1/2)(A1 x W x W + W x A1 x W + W x W x A1) with the 1D
// matrices W = diag(w) and A1 = D^T W D, so that in the bubble basis
// G_ref = (1/2)(Kb x Mb x Mb + Mb x Kb x Mb + Mb x Mb x Kb), Mb = B1^T W B1,
// Kb = B1^T A1 B1 (interior rows and columns).
static std::vector<double> bubble_basis(const sem_handle *h, int &K,
                                        CoarseTab *tab = nullptr) {
  const int N = h->N, n1 = h->n1, m = N - 1, q1 = std::min(2, N - 2) + 1;
  K = q1 * q1 * q1;
  std::vector<double> B1((size_t)m * q1), B((size_t)m * m * m * K);
  for (int i = 0; i < m; ++i) {
    const double x = h->ref.xi[i + 1];
    const double P[3] = {1.0, x, 0.5 * (3.0 * x * x - 1.0)};
    for (int a = 0; a < q1; ++a) B1[(size_t)i * q1 + a] = (1.0 - x * x) * P[a];
  }
  std::vector<double> Mb((size_t)q1 * q1, 0.0), Kb((size_t)q1 * q1, 0.0);
  for (int a = 0; a < q1; ++a)
    for (int b = 0; b < q1; ++b) {
      double mm = 0.0, kk = 0.0;
      for (int i = 0; i < m; ++i)
        mm += B1[(size_t)i * q1 + a] * h->ref.w[i + 1] * B1[(size_t)i * q1 + b];
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          double a1 = 0.0;  // (D^T W D)[i+1][j+1]
          for (int r = 0; r < n1; ++r)
            a1 += h->ref.D[(size_t)r * n1 + i + 1] * h->ref.w[r] *
                  h->ref.D[(size_t)r * n1 + j + 1];
          kk += B1[(size_t)i * q1 + a] * a1 * B1[(size_t)j * q1 + b];
        }
      Mb[(size_t)a * q1 + b] = mm;
      Kb[(size_t)a * q1 + b] = kk;
    }
  std::vector<double> Gr((size_t)K * K);
  for (int c = 0; c < q1; ++c)
    for (int b = 0; b < q1; ++b)
      for (int a = 0; a < q1; ++a)
        for (int c2 = 0; c2 < q1; ++c2)
          for (int b2 = 0; b2 < q1; ++b2)
            for (int a2 = 0; a2 < q1; ++a2) {
              const double ma = Mb[a * q1 + a2], mb = Mb[b * q1 + b2],
                           mc = Mb[c * q1 + c2], ka = Kb[a * q1 + a2],
                           kb = Kb[b * q1 + b2], kc = Kb[c * q1 + c2];
              Gr[(size_t)(a + q1 * (b + q1 * c)) * K + a2 + q1 * (b2 + q1 * c2)] =
                  0.5 * (ka * mb * mc + ma * kb * mc + ma * mb * kc);
            }
  const std::vector<double> Mr = small_inverse(Gr, K);
  std::vector<double> sc(K);
  for (int k = 0; k < K; ++k) sc[k] = std::sqrt(Mr[(size_t)k * K + k]);
  if (tab != nullptr) {
    *tab = CoarseTab{};
    for (int i = 0; i < m; ++i)
      for (int a = 0; a < q1; ++a) tab->B1[i][a] = (float)B1[(size_t)i * q1 + a];
    for (int k = 0; k < K; ++k) tab->sc[k] = (float)sc[k];
  }
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i)
        for (int c = 0; c < q1; ++c)
          for (int b = 0; b < q1; ++b)
            for (int a = 0; a < q1; ++a)
              B[((size_t)(i + m * (j + m * k))) * K + a + q1 * (b + q1 * c)] =
                  B1[(size_t)i * q1 + a] * B1[(size_t)j * q1 + b] *
                  B1[(size_t)k * q1 + c] * sc[a + q1 * (b + q1 * c)];
  return B;
}

// every element's kappa features as a network input row (BF16, zero padding)
__global__ void k_kfeat_rows(int64_t E, const float *__restrict__ kf,
                             uint16_t *__restrict__ X, int ldx) {
  const int64_t e = blockIdx.x;
  for (int q = threadIdx.x; q < ldx; q += blockDim.x)
    X[e * ldx + q] = q < 8 ? f32_to_bf16(kf[e * 8 + q]) : (uint16_t)0;
}

static void kappa_features(const sem_handle *h, DevBuf &kfeat, DevBuf &invkh) {
  kfeat.alloc(h->E * 8 * 4);
  invkh.alloc(h->E * 4);
  hipLaunchKernelGGL(k_kfeat, dim3((unsigned)((h->E + 255) / 256)), dim3(256), 0,
                     0, h->E, h->kvert.as<double>(), elem_size(h),
                     kfeat.as<float>(), invkh.as<float>());
  SEM_HIP(hipGetLastError());
}

static void ensure_learn(sem_handle *h) {
  if (h->learn != nullptr) return;
  Learn *L = new Learn();
  try {
    const int m = h->N - 1;
    L->ni = m * m * m;
    std::vector<double> Bd = bubble_basis(h, L->K, &L->tab);
    const int kp = L->K * (L->K + 1) / 2;
    L->ldx = 16;                    // 8 features, zero padding
    L->ldo = kp > 16 ? kp : 16;
    L->Bd.alloc(Bd.size() * 8);
    SEM_HIP(hipMemcpy(L->Bd.p, Bd.data(), Bd.size() * 8, hipMemcpyHostToDevice));
    L->Sc.alloc((size_t)L->K * 4);
    SEM_HIP(hipMemcpy(L->Sc.p, L->tab.sc, (size_t)L->K * 4, hipMemcpyHostToDevice));
    L->Ml.alloc((size_t)h->E * kp * 4);
    L->cG.alloc((size_t)h->nG * 4);
    SEM_HIP(hipMemset(L->cG.p, 0, (size_t)h->nG * 4));  // faces stay zero
    L->cL.alloc((size_t)h->nL * 4);
    L->ep.alloc((size_t)h->E * 2 * sizeof(double));
    L->O.alloc((size_t)h->E * L->ldo * 4);
    L->exact_damp_dev.alloc(sizeof(float));
    kappa_features(h, L->kfeat, L->invkh);
    L->Xk.alloc((size_t)h->E * L->ldx * 2);
    hipLaunchKernelGGL(k_kfeat_rows, dim3((unsigned)h->E), dim3(64), 0, 0, h->E,
                       L->kfeat.as<float>(), L->Xk.as<uint16_t>(), L->ldx);
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipDeviceSynchronize());
  } catch (...) {
    delete L;
    throw;
  }
  h->learn = L;
}

void drop_graphs(sem_handle *h);

// (re)compute the element operators M_e from the attached network when it
// or its parameters changed (outside any graph capture); exact operators
// never change
void learn_refresh(sem_handle *h) {
  Learn *L = h->learn;
  if (L == nullptr || L->exact || h->net == nullptr) return;
  if (L->mnet == h->net && L->mver == mlp_version(h->net)) return;
  sem_mlp *net = h->net;
  int ldx_net = mlp_padded_inputs(net);
  if (ldx_net != L->ldx) fail(SEM_ERR_STATE, "learned correction: input width");
  mlp_forward(net, L->Xk.as<uint16_t>(), L->ldx, (int)h->E, L->O.as<float>(),
              L->ldo, 0);
  hipLaunchKernelGGL(k_factor_to_M, dim3((unsigned)h->E), dim3(256), 0, 0, h->E,
                     L->K, L->O.as<float>(), L->ldo, L->invkh.as<float>(),
                     L->Ml.as<float>());
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipDeviceSynchronize());
  L->mnet = h->net;
  L->mver = mlp_version(h->net);
}

bool learn_active(const sem_handle *h) {
  return h->learn != nullptr && (h->learn->exact || h->net != nullptr);
}

double learn_damping(const sem_handle *h) {
  return h->learn->exact ? h->learn->exact_damping : mlp_damping(h->net);
}

double learn_ref_rate(const sem_handle *h) {
  return h->learn->exact ? 0.0 : mlp_ref_rate(h->net);
}

void learn_attach(sem_handle *h, sem_mlp *net) {
  drop_graphs(h);
  if (h->learn) h->learn->exact = false;
  if (net == nullptr) {
    h->net = nullptr;
    return;
  }
  check_net(h, net);
  ensure_learn(h);
  h->net = net;
  h->learn->mnet = nullptr;  // recompute M_e for this network
  learn_refresh(h);
}

void learn_apply(sem_handle *h, const void *r, bool f32, hipStream_t s) {
  if (!learn_active(h))
    fail(SEM_ERR_STATE, "learned correction: no network attached");
  Learn *L = h->learn;
  if (f32)
    launch_coarse_apply<float, true>(h, L, (const float *)r, L->cG.as<float>(), s);
  else
    launch_coarse_apply<double, true>(h, L, (const double *)r, L->cG.as<float>(),
                                      s);
}

// flexible CG: z (holding dinv o r) += c(r) on the element interiors, and
// the element terms of (r, c) and (c, w) into epart ([2][E], learn_epart)
void learn_apply_fused(sem_handle *h, const void *r, void *z, const void *wL,
                       bool f32, hipStream_t s) {
  if (!learn_active(h))
    fail(SEM_ERR_STATE, "learned correction: no network attached");
  Learn *L = h->learn;
  if (f32)
    launch_coarse_apply<float, true, true>(h, L, (const float *)r, nullptr, s,
                                           (float *)z, (const float *)wL,
                                           L->ep.as<double>());
  else
    launch_coarse_apply<double, true, true>(h, L, (const double *)r, nullptr, s,
                                            (double *)z, (const double *)wL,
                                            L->ep.as<double>());
}

double *learn_epart(sem_handle *h) { return h->learn ? h->learn->ep.as<double>() : nullptr; }

// the correction on unique nodes (zero off the element interiors)
float *learn_cg(sem_handle *h) { return h->learn ? h->learn->cG.as<float>() : nullptr; }

// z_L = dinv o r_L + c_L on continuous E-vectors (FP64), for
// sem_precond_apply: the coarse correction lives on element-interior nodes,
// each of which has a single copy, and is zero on the faces
__global__ void k_precond_learned_local(int64_t nL, const int32_t *__restrict__ l2g,
                                        const uint8_t *__restrict__ bmask,
                                        const double *__restrict__ dinv,
                                        const float *__restrict__ cL,
                                        const double *__restrict__ r,
                                        double *__restrict__ z) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  z[l] = bmask[l] ? 0.0 : dinv[l2g[l]] * r[l] + (double)cL[l];
}

void learn_precond_local(sem_handle *h, const double *r, double *z, hipStream_t s) {
  if (!learn_active(h))
    fail(SEM_ERR_STATE, "learned correction: no network attached");
  Learn *L = h->learn;
  learn_refresh(h);
  launch_coarse_apply<double, false>(h, L, r, L->cL.as<float>(), s);
  hipLaunchKernelGGL(k_precond_learned_local, dim3((unsigned)((h->nL + 255) / 256)),
                     dim3(256), 0, s, h->nL, h->l2g.as<int32_t>(),
                     h->bmask.as<uint8_t>(), h->dinv_G.as<double>(),
                     L->cL.as<float>(), r, z);
  SEM_HIP(hipGetLastError());
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

template <int N1>
static void launch_coarse_exact_n(const sem_handle *h, const Learn *L, double *U,
                                  double *W, double *Mex, hipStream_t s) {
  constexpr int NT = N1 * N1 <= 64 ? 64 : 128;
  hipLaunchKernelGGL((k_coarse_exact<N1, NT>), dim3((unsigned)h->E), dim3(NT), 0, s,
                     h->E, h->G64.as<double>(), h->D64.as<double>(),
                     L->Bd.as<double>(), L->K, U, W, h->kvert.as<double>(),
                     elem_size(h), Mex);
}

// exact normalised coarse inverses of every element into Mex [E][K][K]
static void coarse_exact(const sem_handle *h, const Learn *L, double *Mex,
                         hipStream_t s) {
  DevBuf U, W;
  const size_t n = (size_t)h->E * h->n1 * h->n1 * h->n1 * 8;
  U.alloc(n);
  W.alloc(n);
  switch (h->N) {
    case 2: launch_coarse_exact_n<3>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    case 3: launch_coarse_exact_n<4>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    case 4: launch_coarse_exact_n<5>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    case 5: launch_coarse_exact_n<6>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    case 6: launch_coarse_exact_n<7>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    case 7: launch_coarse_exact_n<8>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    case 8: launch_coarse_exact_n<9>(h, L, U.as<double>(), W.as<double>(), Mex, s); break;
    default: fail(SEM_ERR_ARG, "coarse layout: N must be in 2..8");
  }
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipStreamSynchronize(s));
}

int learn_coarse_exact(sem_handle *h, double *M, hipStream_t s) {
  if (h->N < 2 || h->N > 8) fail(SEM_ERR_ARG, "coarse layout: N must be in 2..8");
  if (M == nullptr) fail(SEM_ERR_ARG, "coarse layout: null output");
  if (h->has_mass) fail(SEM_ERR_STATE, "coarse layout: mesh has a mass term");
  ensure_learn(h);
  coarse_exact(h, h->learn, M, s);
  return h->learn->K;
}

// attach the exact element coarse inverses (no network) with the given
// damping: the correction the network is trained to imitate
void learn_attach_exact(sem_handle *h, double damping) {
  drop_graphs(h);
  check_mesh(h);
  ensure_learn(h);
  Learn *L = h->learn;
  DevBuf Mex;
  Mex.alloc((size_t)h->E * L->K * L->K * 8);
  coarse_exact(h, L, Mex.as<double>(), 0);
  hipLaunchKernelGGL(k_exact_to_M, dim3((unsigned)h->E), dim3(256), 0, 0, h->E,
                     L->K, Mex.as<double>(), L->invkh.as<float>(), L->Ml.as<float>());
  SEM_HIP(hipGetLastError());
  const float f = (float)damping;
  SEM_HIP(hipMemcpy(L->exact_damp_dev.p, &f, sizeof f, hipMemcpyHostToDevice));
  SEM_HIP(hipDeviceSynchronize());
  h->net = nullptr;
  L->exact = true;
  L->exact_damping = damping;
  L->mnet = nullptr;
}

// snapshot-recording FP64 Jacobi-PCG (solver.hip)
int solve_with_snapshots(sem_handle *h, const double *bL, double *xL, double rtol,
                         int every, int max_snaps, double *xs, double *rs,
                         int *iters, hipStream_t caller);

void learn_train(sem_handle *h, sem_mlp *net, const double *const *bL, int nrhs,
                 const sem_train_opts *o, sem_train_report *rep,
                 hipStream_t caller) {
  check_net(h, net);
  if (nrhs < 1 || bL == nullptr) fail(SEM_ERR_ARG, "train: need right-hand sides");
  if (o->n_pairs < 1 || o->snapshot_every < 1 || o->max_snapshots < 1 ||
      o->epochs < 1 || o->batch < 1 || !(o->lr > 0) || !(o->solve_rtol > 0))
    fail(SEM_ERR_ARG, "train: invalid options");
  if (mlp_padded_inputs(net) != 16)
    fail(SEM_ERR_ARG, "train: the coarse layout takes 8 inputs");
  ensure_learn(h);
  Learn *L = h->learn;
  const int ldx = L->ldx, K = L->K, nt = 2 * K;
  const int64_t nG = h->nG;
  auto t0 = std::chrono::steady_clock::now();

  DevBuf xs, rs, xL, Xd, Td, ps, pe, Xb, Tb, idx, Mex;
  xs.alloc((size_t)o->max_snapshots * nG * 8);
  rs.alloc((size_t)o->max_snapshots * nG * 8);
  xL.alloc(h->nL * 8);
  Xd.alloc((size_t)o->n_pairs * ldx * 2);
  SEM_HIP(hipMemset(Xd.p, 0, (size_t)o->n_pairs * ldx * 2));
  Td.alloc((size_t)o->n_pairs * nt * 4);
  Mex.alloc((size_t)h->E * K * K * 8);
  coarse_exact(h, L, Mex.as<double>(), 0);
  {
    int64_t np = 0, steps = 0;
    int n_in = 0, H = 0, n_out = 0;
    mlp_info(net, &n_in, &H, &n_out, &np, &steps);
    if (steps == 0) {
      // a network that has never been trained starts from the identity
      // factor: output bias = packed identity (in the scaled basis the
      // reference element's coarse inverse has unit diagonal), output
      // weights scaled down so that the start is close to it
      std::vector<float> th((size_t)np);
      mlp_get_params(net, th.data(), np);
      const int64_t w3 = (int64_t)H * n_in + H + (int64_t)H * H + H;
      for (int64_t q = 0; q < (int64_t)n_out * H; ++q) th[w3 + q] *= 0.01f;
      float *b3 = th.data() + w3 + (int64_t)n_out * H;
      for (int q = 0; q < n_out; ++q) b3[q] = 0.f;
      for (int i = 0; i < K; ++i) b3[i * (i + 1) / 2 + i] = 1.f;
      mlp_set_params(net, th.data(), np);
    }
  }
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
    // half the pairs take a random unit direction instead of the residual's
    std::vector<int32_t> hiso(want);
    std::vector<double> hyr((size_t)want * K, 0.0);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int p = 0; p < want; ++p) {
      hiso[p] = (int32_t)(rng() & 1);
      if (!hiso[p]) continue;
      double ss = 0.0;
      for (int k = 0; k < K; ++k) {
        const double v = nd(rng);
        hyr[(size_t)p * K + k] = v;
        ss += v * v;
      }
      const double inv = ss > 0.0 ? 1.0 / std::sqrt(ss) : 0.0;
      for (int k = 0; k < K; ++k) hyr[(size_t)p * K + k] *= inv;
    }
    DevBuf iso, yr;
    iso.alloc((size_t)want * 4);
    yr.alloc(hyr.size() * 8);
    SEM_HIP(hipMemcpy(iso.p, hiso.data(), (size_t)want * 4, hipMemcpyHostToDevice));
    SEM_HIP(hipMemcpy(yr.p, hyr.data(), hyr.size() * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_coarse_pairs, dim3(want), dim3(64), 0, 0, want,
                       ps.as<int32_t>(), pe.as<int32_t>(), nG, h->n1,
                       h->l2g.as<int32_t>(), rs.as<double>(), L->Bd.as<double>(),
                       K, L->ni, Mex.as<double>(), L->kfeat.as<float>(),
                       iso.as<int32_t>(), yr.as<double>(),
                       Xd.as<uint16_t>() + (int64_t)built * ldx, ldx,
                       Td.as<float>() + (int64_t)built * nt);
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipDeviceSynchronize());  // iso, yr are freed at scope end
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
      sum += mlp_loss_grad_factor(net, Xb.as<uint16_t>(), ldx, Tb.as<float>(), K,
                                  B, true, s);
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
  // training right-hand side to 1e-6 is compared with Jacobi-PCG for the
  // damping values 1, 0.75, 0.5, 0.25 (an exact network reproduces the
  // element coarse correction, for which 1 is natural); the best one is
  // kept if it needs fewer iterations than Jacobi, else the correction is
  // disabled (damping 0).
  sem_mlp *prev = h->net;
  const bool prev_exact = L->exact;
  const double prev_exact_d = L->exact_damping;
  const double rate = rate_n ? rate_sum / rate_n : 0.0;
  mlp_set_damping(net, 1.0, 0.0);  // no progress check while validating
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
  const double cand[4] = {1.0, 0.75, 0.5, 0.25};
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
  if (prev_exact)
    learn_attach_exact(h, prev_exact_d);
  else
    learn_attach(h, prev);
  auto t3 = std::chrono::steady_clock::now();
  if (rep) {
    rep->pairs = built;
    rep->epochs = o->epochs;
    rep->snapshots = total_snaps;
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
