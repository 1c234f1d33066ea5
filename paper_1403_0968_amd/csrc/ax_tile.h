// Element routine of the local stiffness action w = D^T G D u (paper
// section 4.2.1), shared by the operator kernels and the element-local
// solves of the learned correction.
//
// One thread per (i,j) column of an element holds the n1 values along k in
// registers (the t-direction contractions never leave registers); the r- and
// s-direction contractions read the current k-slice from LDS (row pitch
// n1+1, so the 8 distinct rows a wave reads at once sit in different banks).
// All loads of an element (its u column and the 6 n1 geometric factors of
// the column) are issued before any arithmetic.  Storage/compute types:
// FP64 (double everywhere), FP32, and BF16 (u and G bfloat16, D, arithmetic
// and w FP32; at n1 = 8 the BF16 factors are stored column-contiguous
// [E][6][n1^2][n1] and the BF16 input is read in 16-byte rows and
// redistributed through LDS).  GATHER = true reads u from a unique-node
// vector through the closed-form box numbering.  MASS = true adds the lumped
// mass term H o u (H = alpha(X) B, one value per local node in the storage
// type of G, natural [E][n1^3] layout: a wave's load of one k-slice is
// contiguous).
#pragma once

#include "common.h"
#include "sem_internal.h"

namespace sem {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class P> __device__ inline auto ld_stream(P p) {
  return __builtin_nontemporal_load(p);
}

// a double moved across the lanes of a wave by a DPP pattern (both halves)
template <int CTRL> __device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// the value of lane `lane` of a wave
__device__ inline double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// LDS row pitch of the slice stacks: n1 + 1 (the 8 distinct rows a wave
// reads at once sit in different banks), or 12 for FP32 arithmetic at n1 =
// 8, where the r-direction rows are read as two 16-byte vectors: 16-byte
// aligned rows whose 8 starts 48 bytes apart cover all 32 banks once
template <int N1, class TC> constexpr int ax_pad() {
  return (N1 == 8 && sizeof(TC) == 4) ? 12 : N1 + 1;
}

template <int N1, class TC = double> constexpr int lds_words(int epb) {
  return 3 * epb * N1 * N1 * ax_pad<N1, TC>();
}

// Workgroup shape of the operator kernels per order and value size (timed on
// the 16.8M-node meshes at every order, and again over 2-4 shapes per order
// with and without the load predicate and the non-temporal hint; every
// choice below is the fastest or within 1.5 % of it).  FP64: elements per workgroup chosen
// so that EPB n1^2 fills whole waves (n1 = 8: four elements, 256 threads),
// and the factors are read with non-temporal loads except at n1 = 2, 3, 5,
// where one factor column is a short piece of a cache line and the
// non-temporal hint makes the neighbouring pieces miss again.  FP32 / BF16:
// 64-thread workgroups.  PRED: the loads carry the thread's element
// predicate instead of reading a valid stand-in element (FP64 at n1 = 7 and
// 9, where the unpredicated loads were 5-7 % slower; elsewhere they are
// faster, by 12 % at n1 = 2 and 16 % at n1 = 3).
template <int N1, int BYTES> struct OpShape {
  static constexpr int NP = N1 * N1;
  static constexpr int EPB64 = N1 == 2 ? 64 : N1 == 3 ? 7 : N1 == 4 ? 4
                               : N1 == 5 ? 5 : N1 == 6 ? 7 : N1 == 7 ? 5
                               : N1 == 8 ? 4 : 3;
  static constexpr int EPB = BYTES == 8 ? EPB64 : ((64 / NP) > 0 ? 64 / NP : 1);
  static constexpr int THREADS = EPB * NP;
  static constexpr bool NTG = BYTES != 8 || !(N1 == 2 || N1 == 3 || N1 == 5);
  static constexpr bool PRED = BYTES == 8 && (N1 == 7 || N1 == 9);
};

// Apply the operator to elements e0 .. e0 + EPB - 1 (those < E) with the
// threads t = 0 .. of one workgroup; threads t >= EPB n1^2 only join the
// barriers.  smem holds 3 EPB n1^2 (n1+1) values of TC (8-byte aligned).
// EDOT = true also stores the element energy edot[e] = u_e^T w_e in FP64,
// summed in an order fixed by the node indices alone (each (i, j) column
// over k, then, at n1 = 8, the 64 column sums in registers by a fixed
// pattern over the lanes c = i + 8 j, otherwise the columns of a row j over
// i and then the rows over j), so that every tile shape gives the same bits.  Inside the solvers u is the
// search direction p, which vanishes on Dirichlet nodes, and the sum of the
// element energies is (p, A p) of the assembled operator.
template <int N1, int EPB, class TU, class TG, class TW, class TC, bool GATHER,
          bool NTW, bool MASS = false, bool NTG = true, bool EDOT = false,
          bool PRED = false>
__device__ __forceinline__ void ax_tile(int t, int64_t e0, int64_t E,
                                        const TC *__restrict__ D_,
                                        const TG *__restrict__ G_,
                                        const TU *__restrict__ u_,
                                        TW *__restrict__ w_,
                                        const Box *__restrict__ box,
                                        TC *__restrict__ smem,
                                        const TG *__restrict__ H_ = nullptr,
                                        double *__restrict__ edot_ = nullptr,
                                        const int32_t *__restrict__ stop = nullptr) {
  // every array is global memory (the batched kernel reads these pointers
  // from a descriptor, where their address space is not known)
  const gp<const TC> D = (gp<const TC>)D_;
  const gp<const TG> G = (gp<const TG>)G_;
  const gp<const TU> u = (gp<const TU>)u_;
  const gp<TW> w = (gp<TW>)w_;
  const gp<const TG> H = (gp<const TG>)H_;
  const gp<double> edot = (gp<double>)edot_;
  constexpr int NP = N1 * N1, N3 = N1 * NP, PAD = ax_pad<N1, TC>();
  // FP32 arithmetic at n1 = 8: the rows (k, j, 0..7) of s_u and s_r are
  // read as two 16-byte vectors
  constexpr bool VROW = PAD == 12;
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  constexpr int SL = N1 * N1 * PAD;  // one element's slice stack
  // n1 = 8: one element per wave (t is the thread index in the workgroup),
  // so the element index and the gather's box arithmetic are wave-uniform
  const int el = NP == 64 ? __builtin_amdgcn_readfirstlane(t / NP) : t / NP;
  const bool lane_ok = el < EPB;
  const int elc = lane_ok ? el : 0;
  const int c = t - el * NP;
  const int i = c % N1, j = c / N1;
  const int64_t e = e0 + el;
  const bool act = lane_ok && e < E;
  const int64_t base = e * N3 + c;
  // loads read element ed: e itself, or the workgroup's first element
  // (always < E) for threads without an element, so that no load needs a
  // predicate; only the stores are guarded.  PRED = true keeps a predicate
  // on every load instead (lanes without an element read nothing)
  const int64_t ed = act ? e : e0;
  const bool ld_on = !PRED || act;
  const int64_t based = ed * N3 + c;
  TC *s_u = smem + (0 * EPB + elc) * SL;
  TC *s_r = smem + (1 * EPB + elc) * SL;
  TC *s_s = smem + (2 * EPB + elc) * SL;
#define AX_IDX(k, jj, ii) (((k) * N1 + (jj)) * PAD + (ii))
  // n1 = 8: an element is one whole wave with its own slice stack, so the
  // phases of the element need only a wave-level barrier
  auto phase_sync = [] {
    if constexpr (NP == 64)
      wave_lds_sync();
    else
      __syncthreads();
  };

  constexpr bool VEC16 = sizeof(TG) == 2 && N1 == 8;  // BF16 column layout
  constexpr bool VECU = sizeof(TU) == 2 && N1 == 8 && !GATHER;
  TU ucol[N1];
  u32x4 urow = {0u, 0u, 0u, 0u};
  if constexpr (VECU) {
    // lane c reads the 16-byte row (k, j) = (c / 8, c % 8) of the element
    urow = *(gp<const u32x4>)(u + ed * N3 + 8 * c);
  } else if constexpr (GATHER) {
    // the column's global (x, y) offset and the element's first z
    // coordinate; a coordinate E_d N of a periodic direction wraps to 0
    const ElemXYZ c3 = box_elem(*box, (uint32_t)ed);
    const uint32_t gx = wrap_coord(c3.x * (uint32_t)(N1 - 1) + i, box->Gx);
    const uint32_t gy = wrap_coord(c3.y * (uint32_t)(N1 - 1) + j, box->Gy);
    const int64_t gxy = (int64_t)gx + (int64_t)box->Gx * gy;
    const uint32_t gz0 = c3.z * (uint32_t)(N1 - 1);
    const int64_t Gxy = box->Gxy;
    // gz0 + k < G_z below the element's last z node: only that one wraps
    const int64_t g0 = gxy + Gxy * gz0;
#pragma unroll
    for (int k = 0; k < N1 - 1; ++k) ucol[k] = ld_on ? u[g0 + Gxy * k] : TU(0);
    ucol[N1 - 1] = ld_on ? u[gxy + Gxy * wrap_coord(gz0 + N1 - 1, box->Gz)] : TU(0);
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) ucol[k] = ld_on ? u[based + k * NP] : TU(0);
  }
  TG g[6][N1];
  if constexpr (VEC16) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const u32x4 v =
          __builtin_nontemporal_load((gp<const u32x4>)(G + ed * 6 * N3 + q * N3 + 8 * c));
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        g[q][2 * h] = (TG)(wv[h] & 0xffffu);
        g[q][2 * h + 1] = (TG)(wv[h] >> 16);
      }
    }
  } else {
    const gp<const TG> Ge = G + ed * 6 * N3 + c;
#pragma unroll
    for (int k = 0; k < N1; ++k)
#pragma unroll
      for (int q = 0; q < 6; ++q)
        g[q][k] = !ld_on ? TG(0)
                  : NTG  ? ld_stream(Ge + q * N3 + k * NP)
                         : Ge[q * N3 + k * NP];
  }

  TG hm[MASS ? N1 : 1];
  if constexpr (MASS) {
#pragma unroll
    for (int k = 0; k < N1; ++k) hm[k] = ld_on ? ld_stream(H + based + k * NP) : TG(0);
  }
  // every load above is issued before anything below: without the fence
  // the scheduler may wait for u (to store it into LDS) before it issues the
  // factor loads, which halves the bytes in flight (165 -> 201 us, FP64,
  // 32^3, N = 7)
  __builtin_amdgcn_sched_barrier(0);
  // a solver's done flag (uniform over the workgroup) is read only now, with
  // the element's loads already in flight: waiting for it before them put a
  // memory round trip in front of every workgroup
  if (stop != nullptr && *stop != 0) return;

  TC uc[N1];
  if constexpr (VECU) {
    const uint32_t wv[4] = {urow.x, urow.y, urow.z, urow.w};
    if (lane_ok) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        s_u[AX_IDX(c / 8, c % 8, 2 * h)] = Cvt<TU, TC>::ld((TU)(wv[h] & 0xffffu));
        s_u[AX_IDX(c / 8, c % 8, 2 * h + 1)] = Cvt<TU, TC>::ld((TU)(wv[h] >> 16));
      }
    }
    phase_sync();
#pragma unroll
    for (int k = 0; k < N1; ++k) uc[k] = s_u[AX_IDX(k, j, i)];
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      uc[k] = Cvt<TU, TC>::ld(ucol[k]);
      if (lane_ok) s_u[AX_IDX(k, j, i)] = uc[k];
    }
  }
  // mass term H o u, formed while u is in registers; it starts the output sum
  TC mv[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    if constexpr (MASS)
      mv[k] = Cvt<TG, TC>::ld(hm[k]) * uc[k];
    else
      mv[k] = TC(0);
  }
  TC Di[N1], Dj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    Di[m] = D[i * N1 + m];
    Dj[m] = D[j * N1 + m];
  }
  phase_sync();

  // gradient (r, s from LDS; t from registers) and fluxes, slice by slice
  TC wt[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    TC ur = TC(0), us = TC(0), ut = TC(0);
    TC rowu[VROW ? N1 : 1];
    if constexpr (VROW) {
      const f32x4 a0 = *reinterpret_cast<const f32x4 *>(&s_u[AX_IDX(k, j, 0)]);
      const f32x4 a1 = *reinterpret_cast<const f32x4 *>(&s_u[AX_IDX(k, j, 4)]);
      rowu[0] = a0.x, rowu[1] = a0.y, rowu[2] = a0.z, rowu[3] = a0.w;
      rowu[4] = a1.x, rowu[5] = a1.y, rowu[6] = a1.z, rowu[7] = a1.w;
    }
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      ur += Di[m] * (VROW ? rowu[VROW ? m : 0] : s_u[AX_IDX(k, j, m)]);
      us += Dj[m] * s_u[AX_IDX(k, m, i)];
      ut += D[k * N1 + m] * uc[m];
    }
    const TC g0 = Cvt<TG, TC>::ld(g[0][k]), g1 = Cvt<TG, TC>::ld(g[1][k]),
             g2 = Cvt<TG, TC>::ld(g[2][k]), g3 = Cvt<TG, TC>::ld(g[3][k]),
             g4 = Cvt<TG, TC>::ld(g[4][k]), g5 = Cvt<TG, TC>::ld(g[5][k]);
    if (lane_ok) {
      s_r[AX_IDX(k, j, i)] = g0 * ur + g1 * us + g2 * ut;
      s_s[AX_IDX(k, j, i)] = g1 * ur + g3 * us + g4 * ut;
    }
    wt[k] = g2 * ur + g4 * us + g5 * ut;
  }
  phase_sync();

  // w = D_r^T w_r + D_s^T w_s + D_t^T w_t
  TC DTi[N1], DTj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    DTi[m] = D[m * N1 + i];
    DTj[m] = D[m * N1 + j];
  }
  double cdot = 0.0;  // EDOT: this column's u^T w
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    TC acc = mv[k];
    TC rowr[VROW ? N1 : 1];
    if constexpr (VROW) {
      const f32x4 a0 = *reinterpret_cast<const f32x4 *>(&s_r[AX_IDX(k, j, 0)]);
      const f32x4 a1 = *reinterpret_cast<const f32x4 *>(&s_r[AX_IDX(k, j, 4)]);
      rowr[0] = a0.x, rowr[1] = a0.y, rowr[2] = a0.z, rowr[3] = a0.w;
      rowr[4] = a1.x, rowr[5] = a1.y, rowr[6] = a1.z, rowr[7] = a1.w;
    }
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      acc += DTi[m] * (VROW ? rowr[VROW ? m : 0] : s_r[AX_IDX(k, j, m)]);
      acc += DTj[m] * s_s[AX_IDX(k, m, i)];
      acc += D[m * N1 + k] * wt[m];
    }
    if constexpr (EDOT) cdot += (double)uc[k] * (double)(TW)acc;
    if (act) {
      if constexpr (NTW)
        __builtin_nontemporal_store((TW)acc, w + base + k * NP);
      else
        w[base + k * NP] = (TW)acc;
    }
  }
  if constexpr (EDOT && NP == 64) {
    // n1 = 8: every element is one whole wave (its 64 columns are the lanes
    // of a wave in every tile shape), so the column sums are added in
    // registers: lane exchanges within quads, then mirrored halves of each
    // 8 and 16 lanes (each step adds two equal-sized partial sums, and
    // a + b = b + a, so all lanes of a row hold the same bits), then the
    // four row sums in order
    double v = cdot;
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    const double sum =
        ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
    if (act && c == 0) edot[e] = sum;
  } else if constexpr (EDOT) {
    // s_u is no longer read after the barrier above: it holds the column
    // sums red[c] (c = i + n1 j) and then the row sums red[NP + j]
    double *red = reinterpret_cast<double *>(s_u);
    if (lane_ok) red[c] = cdot;
    __syncthreads();
    if (lane_ok && i == 0) {
      double r = 0.0;
#pragma unroll
      for (int ii = 0; ii < N1; ++ii) r += red[ii + N1 * j];
      red[NP + j] = r;
    }
    __syncthreads();
    if (act && c == 0) {
      double r = 0.0;
#pragma unroll
      for (int jj = 0; jj < N1; ++jj) r += red[NP + jj];
      edot[e] = r;
    }
  }
#undef AX_IDX
}

}  // namespace sem
