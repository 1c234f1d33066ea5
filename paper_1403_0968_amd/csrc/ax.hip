// Local stiffness action w = D^T G D u on hexahedral spectral elements
// (paper section 4.2.1, factored stiffness operator with the G^T G metric
// precomputed per elemental node; section 4.2.2 names it the dominant cost of
// every PCG iteration).
//
// Kernel design for gfx950 (HBM-bound: 64 B per node in FP64 against ~111
// flops per node at N=7):
//   * one thread per (i,j) column of an element, holding the n1 values along
//     k in registers: the t-direction contractions never leave registers;
//   * the r- and s-direction contractions read the current k-slice from LDS
//     (row pitch n1+1 so that the 8 distinct rows a wave reads at once sit in
//     different banks);
//   * the six geometric factors of a slice are read with one fully coalesced
//     load per factor (consecutive lanes, consecutive nodes);
//   * all loads of an element (its u column and the 6 n1 geometric factors of
//     the column) are issued before any arithmetic, so each wave keeps its
//     whole input in flight; the factors are read once per operator
//     application and bypass the caches (non-temporal loads), and so do the
//     outputs of the standalone operator;
//   * u, the r-flux and the s-flux each have their own LDS array; FP64 uses
//     128-thread workgroups, FP32/BF16 64-thread ones (two / one element at
//     n1 = 8).
// Storage/compute type combinations:
//   FP64: u, G, w double; FP32: float everywhere;
//   BF16: u and G bfloat16, D, arithmetic and w in FP32.  At n1 = 8 the BF16
//   factors are stored column-contiguous ([E][6][n1^2][n1]) so that a lane
//   fetches the 8 values of one factor with a single 16-byte load, and the
//   BF16 input is read in 16-byte rows and redistributed through LDS.
// GATHER = true reads u from a unique-node vector through l2g (the Q of the
// assembled operator), used inside the solvers.
#include "common.h"
#include "sem_internal.h"

namespace sem {

template <int N1, int BYTES> struct AxShape {
  static constexpr int NP = N1 * N1;
  // FP64: two 64-lane columns sets per workgroup at N1 = 8; FP32/BF16: one
  static constexpr int TARGET = BYTES == 8 ? 128 : 64;
  static constexpr int EPB = (TARGET / NP) > 0 ? (TARGET / NP) : 1;
  static constexpr int THREADS = EPB * NP;
  static constexpr int N3 = N1 * NP;
  static constexpr int PAD = N1 + 1;
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T> __device__ inline T ld_stream(const T *p) {
  return __builtin_nontemporal_load(p);
}

template <int N1, class TU, class TG, class TW, class TC, bool GATHER, bool NTW>
__global__ void __launch_bounds__((AxShape<N1, sizeof(TC)>::THREADS))
    k_ax(int64_t E, const TC *__restrict__ D, const TG *__restrict__ G,
         const TU *__restrict__ u, TW *__restrict__ w,
         const int32_t *__restrict__ l2g, const int32_t *__restrict__ stop) {
  using S = AxShape<N1, sizeof(TC)>;
  constexpr int NP = S::NP, N3 = S::N3, EPB = S::EPB, PAD = S::PAD;
  __shared__ TC s_u[EPB][N1][N1][PAD];  // u
  __shared__ TC s_r[EPB][N1][N1][PAD];  // r-flux
  __shared__ TC s_s[EPB][N1][N1][PAD];  // s-flux

  if (stop != nullptr && *stop != 0) return;  // uniform: solver finished

  const int t = threadIdx.x;
  const int el = t / NP;
  const int c = t - el * NP;
  const int i = c % N1, j = c / N1;
  const int64_t e = (int64_t)blockIdx.x * EPB + el;
  const bool act = e < E;
  const int64_t base = e * N3 + c;

  // every load of the element is issued before any arithmetic: the u column
  // and all 6 x n1 geometric factors of the column (streamed, read once)
  constexpr bool VEC16 = sizeof(TG) == 2 && N1 == 8;  // BF16 column layout
  constexpr bool VECU = sizeof(TU) == 2 && N1 == 8 && !GATHER;
  TU ucol[N1];
  u32x4 urow = {0u, 0u, 0u, 0u};
  if constexpr (VECU) {
    // lane c reads the 16-byte row (k, j) = (c / 8, c % 8) of the element
    if (act) urow = *reinterpret_cast<const u32x4 *>(u + e * N3 + 8 * c);
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      TU v = TU(0);
      if (act) {
        if constexpr (GATHER)
          v = u[l2g[base + k * NP]];
        else
          v = u[base + k * NP];
      }
      ucol[k] = v;
    }
  }
  TG g[6][N1];
  if constexpr (VEC16) {
    // layout [E][6][n1^2][n1]: the n1 values of one column are contiguous
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (act)
        v = __builtin_nontemporal_load(
            reinterpret_cast<const u32x4 *>(G + e * 6 * N3 + q * N3 + 8 * c));
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        g[q][2 * h] = (TG)(wv[h] & 0xffffu);
        g[q][2 * h + 1] = (TG)(wv[h] >> 16);
      }
    }
  } else {
    const TG *Ge = G + e * 6 * N3 + c;
#pragma unroll
    for (int k = 0; k < N1; ++k)
#pragma unroll
      for (int q = 0; q < 6; ++q)
        g[q][k] = act ? ld_stream(Ge + q * N3 + k * NP) : TG(0);
  }

  TC uc[N1];
  if constexpr (VECU) {
    const uint32_t wv[4] = {urow.x, urow.y, urow.z, urow.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      s_u[el][c / 8][c % 8][2 * h] = Cvt<TU, TC>::ld((TU)(wv[h] & 0xffffu));
      s_u[el][c / 8][c % 8][2 * h + 1] = Cvt<TU, TC>::ld((TU)(wv[h] >> 16));
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N1; ++k) uc[k] = s_u[el][k][j][i];
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      uc[k] = Cvt<TU, TC>::ld(ucol[k]);
      s_u[el][k][j][i] = uc[k];
    }
  }
  TC Di[N1], Dj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    Di[m] = D[i * N1 + m];
    Dj[m] = D[j * N1 + m];
  }
  __syncthreads();

  // gradient (r, s from LDS; t from registers) and fluxes, slice by slice
  TC wt[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    TC ur = TC(0), us = TC(0), ut = TC(0);
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      ur += Di[m] * s_u[el][k][j][m];
      us += Dj[m] * s_u[el][k][m][i];
      ut += D[k * N1 + m] * uc[m];
    }
    const TC g0 = Cvt<TG, TC>::ld(g[0][k]), g1 = Cvt<TG, TC>::ld(g[1][k]),
             g2 = Cvt<TG, TC>::ld(g[2][k]), g3 = Cvt<TG, TC>::ld(g[3][k]),
             g4 = Cvt<TG, TC>::ld(g[4][k]), g5 = Cvt<TG, TC>::ld(g[5][k]);
    s_r[el][k][j][i] = g0 * ur + g1 * us + g2 * ut;
    s_s[el][k][j][i] = g1 * ur + g3 * us + g4 * ut;
    wt[k] = g2 * ur + g4 * us + g5 * ut;
  }
  __syncthreads();

  // w = D_r^T w_r + D_s^T w_s + D_t^T w_t
  TC DTi[N1], DTj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    DTi[m] = D[m * N1 + i];
    DTj[m] = D[m * N1 + j];
  }
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    TC acc = TC(0);
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      acc += DTi[m] * s_r[el][k][j][m];
      acc += DTj[m] * s_s[el][k][m][i];
      acc += D[m * N1 + k] * wt[m];
    }
    if (act) {
      if constexpr (NTW)
        __builtin_nontemporal_store((TW)acc, w + base + k * NP);
      else
        w[base + k * NP] = (TW)acc;
    }
  }
}

template <int N1>
static void launch_n(int prec, int64_t E, const void *D, const void *G,
                     const void *u, void *w, const int32_t *l2g,
                     const int32_t *stop, hipStream_t s) {
  using S8 = AxShape<N1, 8>;
  using S4 = AxShape<N1, 4>;
  const int epb = prec == SEM_FP64 ? S8::EPB : S4::EPB;
  const int threads = prec == SEM_FP64 ? S8::THREADS : S4::THREADS;
  const int64_t blocks = (E + epb - 1) / epb;
  if (blocks == 0) return;
  dim3 grid((unsigned)blocks), block(threads);
  const bool gather = l2g != nullptr;
  if (prec == SEM_FP64) {
    if (gather)
      hipLaunchKernelGGL((k_ax<N1, double, double, double, double, true, false>), grid,
                         block, 0, s, E, (const double *)D, (const double *)G,
                         (const double *)u, (double *)w, l2g, stop);
    else
      hipLaunchKernelGGL((k_ax<N1, double, double, double, double, false, true>),
                         grid, block, 0, s, E, (const double *)D,
                         (const double *)G, (const double *)u, (double *)w, l2g,
                         stop);
  } else if (prec == SEM_FP32) {
    if (gather)
      hipLaunchKernelGGL((k_ax<N1, float, float, float, float, true, false>), grid,
                         block, 0, s, E, (const float *)D, (const float *)G,
                         (const float *)u, (float *)w, l2g, stop);
    else
      hipLaunchKernelGGL((k_ax<N1, float, float, float, float, false, true>), grid,
                         block, 0, s, E, (const float *)D, (const float *)G,
                         (const float *)u, (float *)w, l2g, stop);
  } else {
    // BF16 geometric factors.  Standalone: bf16 input; inside solvers the
    // FP32 unique vector is gathered directly.
    if (gather)
      hipLaunchKernelGGL((k_ax<N1, float, uint16_t, float, float, true, false>), grid,
                         block, 0, s, E, (const float *)D, (const uint16_t *)G,
                         (const float *)u, (float *)w, l2g, stop);
    else
      hipLaunchKernelGGL((k_ax<N1, uint16_t, uint16_t, float, float, false, true>),
                         grid, block, 0, s, E, (const float *)D,
                         (const uint16_t *)G, (const uint16_t *)u, (float *)w,
                         l2g, stop);
  }
}

void launch_ax(int N, int prec, int64_t E, const void *D, const void *G,
               const void *u, void *w, const int32_t *l2g, const int32_t *stop,
               hipStream_t s) {
  switch (N) {
    case 1: launch_n<2>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 2: launch_n<3>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 3: launch_n<4>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 4: launch_n<5>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 5: launch_n<6>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 6: launch_n<7>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 7: launch_n<8>(prec, E, D, G, u, w, l2g, stop, s); break;
    case 8: launch_n<9>(prec, E, D, G, u, w, l2g, stop, s); break;
    default: fail(SEM_ERR_ARG, "sem_ax: N must be in 1..8");
  }
  SEM_HIP(hipGetLastError());
}

}  // namespace sem
