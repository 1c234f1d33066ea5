// DG volume term of the 2D shallow-water equations (paper section 4.3): for
// every triangle, rhs = Dxw F + Dyw G + S with the nodal fluxes
//   F = (hu, hu^2/h + g h^2/2, hu hv/h), G = (hv, hu hv/h, hv^2/h + g h^2/2),
// source S = (0, -g h B_x, -g h B_y), and on an affine element
//   Dxw F + Dyw G = Drw (rx F + ry G) + Dsw (sx F + sy G).
//
// The two weak derivative matrices are shared by all elements, so the term is
// one dense product [Drw | Dsw] (Np x 2Np) times the stacked metric-weighted
// fluxes (2Np x 3E), plus the nodal source.  It runs on the FP64 matrix
// cores (v_mfma_f64_16x16x4): one wave takes 16 elements as the 16 columns
// of the product, one component at a time; the row tiles cover the Np
// output nodes (padded to 16), the K steps run over the nodes four at a time
// (padded to 4) for Drw and Dsw together.  Lane l supplies the B operand for
// (element l % 16, node 4 step + l / 16): it loads h, hu, hv there and forms
// the fluxes itself, so the operand never passes through LDS.  The A
// operands come from copies of Drw / Dsw that the host stores in the lane
// order of the instruction (entry [(ks NT + t) 64 + l] = row 16 t + l % 16,
// column 4 ks + l / 16, zero-padded): each wave's load of them is 512
// contiguous bytes instead of 16 pieces of 32 bytes (N = 4..8: 44.3, 90.6,
// 118.6, 166.9, 273.0 -> 42.0, 84.7, 108.5, 152.3, 225.2 us).  Output
// element v of lane l is row l / 16 + 4 v of the tile.
// The loads of K step ks + 1 (the lane's state, at a clamped node index, and
// its operator entries) are issued before the products of step ks, so the
// memory latency of one step hides behind the matrix instructions of the
// previous one; per step, all Drw products come first, then all Dsw
// products, so the two updates of one accumulator are 3 NT instructions
// apart.  Timed on the 212,800-element mesh against loading each step's
// operands just before use (with separate Drw / Dsw accumulators from N = 7):
// N = 2..8 20.2, 32.7, 55.4, 103, 129, 209, 313 us -> 17.9, 28.6, 44.1,
// 91.4, 118, 167, 272 us.  The K loop is unrolled completely; at N = 7 the
// kernel is compiled for at least two waves per SIMD (its 166 registers fit
// three; the hint still shapes the schedule).  The
// accumulators stay in ordinary vector registers (the source is compiled
// with the matrix instructions' VGPR form): in the accumulation registers
// the compiler copied the loop-carried ones in and out on every K step of
// a partly unrolled loop (96 copies per two steps at N = 8), and at N = 8
// that copying was what kept the K loop from being unrolled completely
// (N = 6, 8: 79.4, 158.5 -> 74.5, 142.4 us).
// Measured limits: a dependency-free loop of these instructions reaches
// about 48 TFLOP/s on this chip (FP64 FMA on the vector units about 66).
#include "common.h"
#include "sem_internal.h"

namespace sem {

typedef double dg_d4 __attribute__((ext_vector_type(4)));

constexpr int DG_WAVES = 4;  // waves per workgroup, 16 elements each

template <int N> struct DgShape {
  static constexpr int NP = (N + 1) * (N + 2) / 2;
  static constexpr int NT = (NP + 15) / 16;  // output row tiles
  static constexpr int NK = (NP + 3) / 4;    // K steps of four nodes
  static constexpr int WAVES_PER_EU = N == 7 ? 2 : 1;
};

// BLK = false: state, result and bathymetry gradient element-major,
// [E][3][Np] and [E][2][Np]; every load or store of a wave touches 16
// elements x 32 bytes.  BLK = true: blocks of 16 elements, [E/16][3][Np][16]
// and [E/16][2][Np][16] (element fastest), so each of them is 512
// contiguous bytes.
template <int N, bool BLK>
__global__ void __launch_bounds__(64 * DG_WAVES)
    __attribute__((amdgpu_waves_per_eu(DgShape<N>::WAVES_PER_EU)))
    k_dg_volume(int64_t E, const double *__restrict__ Q, double *__restrict__ rhs,
                const double *__restrict__ geo, const double *__restrict__ dB,
                const double *__restrict__ Drw, const double *__restrict__ Dsw,
                double g) {
  using S = DgShape<N>;
  constexpr int NP = S::NP, NT = S::NT, NK = S::NK;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t blk = (int64_t)blockIdx.x * DG_WAVES + wave;
  const int64_t e = blk * 16 + col;
  const bool act = e < E;
  // a wave past the last block has nothing to do (no barrier in this kernel)
  if (BLK && blk * 16 >= E) return;
  // node m of component c of this lane's element (an element of the mesh:
  // lanes past the last element read the block's first one)
  //   element-major: Qe[c NP + m]; blocks: Qe[(c NP + m) 16]
  constexpr int CS = BLK ? 16 : 1;
  const double *Qe = BLK ? Q + blk * 3 * NP * 16 + (act ? col : 0)
                         : Q + (act ? e : 0) * 3 * NP;
  // this lane's A operand entries (row 16 t + col, column 4 ks + kq) are
  // entries (ks NT + t) 64 + lane of the lane-order copies
  const double *Ar = Drw + lane, *As = Dsw + lane;
  double rx = 0.0, sx = 0.0, ry = 0.0, sy = 0.0;
  if (act) {
    rx = geo[4 * e];
    sx = geo[4 * e + 1];
    ry = geo[4 * e + 2];
    sy = geo[4 * e + 3];
  }
  dg_d4 acc[3][NT];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[q][t] = dg_d4{0.0, 0.0, 0.0, 0.0};
  const double hg = 0.5 * g;
  // with the K loop unrolled completely, the depth this lane loads at K step
  // ks is the depth at its output row 16 t + kq + 4 v for ks = 4 t + v: kept
  // for the source term instead of loaded again (N = 4..7: 42.1, 85.0,
  // 109.2, 152.6 -> 39.4, 75.3, 105.5, 144.9 us)
  double hk[NK];
  double qn[3], an[NT], sn[NT];  // operands of the next K step
  auto fetch = [&](int ks) {
    const int m = min(4 * ks + kq, NP - 1);
    qn[0] = Qe[m * CS];
    qn[1] = Qe[(NP + m) * CS];
    qn[2] = Qe[(2 * NP + m) * CS];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      an[t] = Ar[(ks * NT + t) * 64];
      sn[t] = As[(ks * NT + t) * 64];
    }
  };
  fetch(0);
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) {
    const double h = qn[0], hu = qn[1], hv = qn[2];
    hk[ks] = h;
    double ar[NT], as[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ar[t] = an[t];
      as[t] = sn[t];
    }
    if (ks + 1 < NK) fetch(ks + 1);
    // fluxes at node 4 ks + kq of element e (zero beyond Np or the mesh)
    // one reciprocal instead of two divisions; hu v = hv u is formed once
    const double ih = 1.0 / h, u = hu * ih, v = hv * ih, p = hg * h * h;
    const double huv = hu * v;
    const double F[3] = {hu, hu * u + p, huv};
    const double G[3] = {hv, huv, hv * v + p};
    const bool ok = act && 4 * ks + kq < NP;
    double xr[3], xs[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      xr[q] = ok ? rx * F[q] + ry * G[q] : 0.0;
      xs[q] = ok ? sx * F[q] + sy * G[q] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc[q][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[t], xr[q], acc[q][t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        acc[q][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[t], xs[q], acc[q][t], 0, 0, 0);
  }
  if (!act) return;
  double *Re = BLK ? rhs + blk * 3 * NP * 16 + col : rhs + e * 3 * NP;
  const double *Bx = BLK ? dB + blk * 2 * NP * 16 + col : dB + e * 2 * NP;
  const double *By = Bx + NP * CS;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + kq + 4 * v;
      if (r < NP) {
        // r < Np puts 4 t + v below NK; the clamp only keeps the index in
        // range in code for rows r >= Np, which never runs
        const int KS = 4 * t + v < NK ? 4 * t + v : NK - 1;
        const double gh = g * hk[KS];
        Re[r * CS] = acc[0][t][v];
        Re[(NP + r) * CS] = acc[1][t][v] - gh * Bx[r * CS];
        Re[(2 * NP + r) * CS] = acc[2][t][v] - gh * By[r * CS];
      }
    }
}

template <int N>
static void launch_n(const dg_handle *h, const double *Q, double *rhs, bool blocked,
                     hipStream_t s) {
  const int64_t per = 16 * DG_WAVES;
  const int64_t blocks = (h->E + per - 1) / per;
  if (blocks == 0) return;
  if (blocked)
    hipLaunchKernelGGL((k_dg_volume<N, true>), dim3((unsigned)blocks),
                       dim3(64 * DG_WAVES), 0, s, h->E, Q, rhs, h->geo.as<double>(),
                       h->dBb.as<double>(), h->Drw.as<double>(),
                       h->Dsw.as<double>(), h->g);
  else
    hipLaunchKernelGGL((k_dg_volume<N, false>), dim3((unsigned)blocks),
                       dim3(64 * DG_WAVES), 0, s, h->E, Q, rhs, h->geo.as<double>(),
                       h->dB.as<double>(), h->Drw.as<double>(),
                       h->Dsw.as<double>(), h->g);
}

void launch_dg_volume(const dg_handle *h, const double *Q, double *rhs,
                      bool blocked, hipStream_t s) {
  switch (h->N) {
    case 1: launch_n<1>(h, Q, rhs, blocked, s); break;
    case 2: launch_n<2>(h, Q, rhs, blocked, s); break;
    case 3: launch_n<3>(h, Q, rhs, blocked, s); break;
    case 4: launch_n<4>(h, Q, rhs, blocked, s); break;
    case 5: launch_n<5>(h, Q, rhs, blocked, s); break;
    case 6: launch_n<6>(h, Q, rhs, blocked, s); break;
    case 7: launch_n<7>(h, Q, rhs, blocked, s); break;
    case 8: launch_n<8>(h, Q, rhs, blocked, s); break;
    default: fail(SEM_ERR_ARG, "dg: N must be in 1..8");
  }
  SEM_HIP(hipGetLastError());
}


// Host setup: reference operators, affine factors, node coordinates and the
// bathymetry gradient (derivative of B's nodal interpolant), uploaded once.
void dg_device_setup(dg_handle *h, int64_t nv, const double *vx, const double *vy,
                     const int32_t *etov, const double *B, hipStream_t s) {
  const int N = h->N;
  h->ref = make_dg_ref(N);
  const int Np = h->ref.Np;
  h->Np = Np;
  const int64_t E = h->E;
  const std::vector<double> &r = h->ref.r, &sn = h->ref.s;
  std::vector<double> geo(4 * E), X(E * Np), Y(E * Np), dB(E * 2 * Np, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t a = etov[3 * e], b = etov[3 * e + 1], c = etov[3 * e + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
      fail(SEM_ERR_ARG, "dg_setup: element vertex index out of range");
    const double xr = 0.5 * (vx[b] - vx[a]), xs = 0.5 * (vx[c] - vx[a]);
    const double yr = 0.5 * (vy[b] - vy[a]), ys = 0.5 * (vy[c] - vy[a]);
    const double J = xr * ys - xs * yr;
    if (!(J > 0.0) || !std::isfinite(J))
      fail(SEM_ERR_ARG, "dg_setup: elements must be non-degenerate and counterclockwise");
    geo[4 * e] = ys / J;
    geo[4 * e + 1] = -yr / J;
    geo[4 * e + 2] = -xs / J;
    geo[4 * e + 3] = xr / J;
    for (int n = 0; n < Np; ++n) {
      const double la = -0.5 * (r[n] + sn[n]), lb = 0.5 * (1.0 + r[n]), lc = 0.5 * (1.0 + sn[n]);
      X[e * Np + n] = la * vx[a] + lb * vx[b] + lc * vx[c];
      Y[e * Np + n] = la * vy[a] + lb * vy[b] + lc * vy[c];
    }
    if (B != nullptr) {
      const double *Be = B + e * Np;
      for (int n = 0; n < Np; ++n) {
        double br = 0.0, bs = 0.0;
        for (int m = 0; m < Np; ++m) {
          br += h->ref.Dr[n * Np + m] * Be[m];
          bs += h->ref.Ds[n * Np + m] * Be[m];
        }
        dB[e * 2 * Np + n] = geo[4 * e] * br + geo[4 * e + 1] * bs;
        dB[e * 2 * Np + Np + n] = geo[4 * e + 2] * br + geo[4 * e + 3] * bs;
      }
    }
  }
  // Drw, Dsw in the lane order of the matrix instruction, zero-padded
  const int nt = (Np + 15) / 16, nk = (Np + 3) / 4;
  std::vector<double> Ar((size_t)nk * nt * 64, 0.0), As((size_t)nk * nt * 64, 0.0);
  for (int ks = 0; ks < nk; ++ks)
    for (int t = 0; t < nt; ++t)
      for (int l = 0; l < 64; ++l) {
        const int i = 16 * t + l % 16, k = 4 * ks + l / 16;
        if (i < Np && k < Np) {
          Ar[((size_t)ks * nt + t) * 64 + l] = h->ref.Drw[i * Np + k];
          As[((size_t)ks * nt + t) * 64 + l] = h->ref.Dsw[i * Np + k];
        }
      }
  // the same gradient in blocks of 16 elements, [E/16][2][Np][16] (zero
  // padding in the last block)
  const int64_t nb = (E + 15) / 16;
  std::vector<double> dBb((size_t)nb * 2 * Np * 16, 0.0);
  for (int64_t e = 0; e < E; ++e)
    for (int c = 0; c < 2; ++c)
      for (int n = 0; n < Np; ++n)
        dBb[(((size_t)(e / 16) * 2 + c) * Np + n) * 16 + e % 16] =
            dB[((size_t)e * 2 + c) * Np + n];
  auto up = [&](DevBuf &d, const std::vector<double> &v) {
    d.alloc(v.size() * sizeof(double));
    SEM_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
  };
  up(h->geo, geo);
  up(h->dB, dB);
  up(h->dBb, dBb);
  up(h->X, X);
  up(h->Y, Y);
  up(h->Drw, Ar);
  up(h->Dsw, As);
  SEM_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
}

}  // namespace sem
