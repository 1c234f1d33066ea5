// Local stiffness action w = D^T G D u (paper section 4.2.1) with the six
// tensor contractions on the matrix cores: BF16 inputs u and G, FP32
// accumulation, FP32 output.
//
// The derivative matrix cannot simply be rounded to BF16: its rounding error
// does not vanish on smooth inputs (D 1 != 0, D x != 1), which the
// refinement around the operator cannot undo.  It is split instead,
// D = D_hi + D_lo with D_hi = bf16(D) and D_lo = bf16(D - D_hi) (a two-term
// BF16 expansion, relative error ~2^-16), and every contraction runs as two
// accumulating MFMAs.  SPLIT = false keeps only D_hi (the inaccurate
// variant, kept for measurement).
//
// One wave per element, the element padded to 8^3 nodes (n1 <= 8; padded
// entries of u and D are zero), four waves per workgroup, each with its own
// LDS region: the phases of an element are ordered by wave-level barriers,
// so the waves of a workgroup do not wait for each other.  MFMA tile
// 16x16x16 (v_mfma_f32_16x16x16_bf16): lane l = 16 g + r holds A[r][4g + q],
// B[4g + q][r] and C[4g + q][r], q = 0..3.  A length-8 contraction uses a
// block-diagonal operand diag(D, D) so that one MFMA contracts two 8-blocks:
//   t (over k):  C[(b,k)][c']   = sum_m D[k][m] u[m][cb + 16 b + c']
//   r (over i):  C[rho'][(b,i)] = sum_m u[rb + 16 b + rho'][m] D[i][m]
//   s (over j):  C[(b,j)][(h,i)] = sum_m D[j][m] u[kb + 2 b + h][m][i]
// with c = (j,i) and rho = (k,j); two MFMAs (cb, rb, kb) cover the element.
// The transposed contractions use D^T the same way and accumulate w through
// the C operand (r, then s, then t), staged in LDS in [k][j][i] order.  The
// metric step between them (fluxes = G grad u) is FP32 on the VALU, one lane
// per (i,j) column, and the fluxes are rounded to BF16 for the MFMAs.  With a
// mass term the lumped H o u (H = alpha(X) B in BF16) is added in FP32 as the
// result leaves LDS.
#include "ax_tile.h"

namespace sem {

typedef short m16x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

constexpr int MW = 4;  // waves (elements) per workgroup

struct alignas(16) MfmaLds {
  uint16_t u[512];                  // u (BF16), or the high term of its split
  float gr[512], gs[512], gt[512];  // gradients; gr is reused for w
  uint16_t fr[512], fs[512], ft[512];
};
// with the low term of a split input: ul = bf16(u - bf16(u))
struct alignas(16) MfmaLdsSplit : MfmaLds {
  uint16_t ul[512];
};

__device__ inline m16x4 lds4_strided(const uint16_t *p, int stride) {
  m16x4 v;
  v[0] = (short)p[0];
  v[1] = (short)p[stride];
  v[2] = (short)p[2 * stride];
  v[3] = (short)p[3 * stride];
  return v;
}

__device__ inline mf32x4 mfma(m16x4 a, m16x4 b, mf32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Operands of the derivative matrix held by lane l (constant per kernel):
//   fwd[q] = D[r % 8][4 (g % 2) + q], bwd[q] = D[4 (g % 2) + q][r % 8],
// zero off the diagonal blocks (r / 8 != g / 2) and outside n1.
template <int N1>
__device__ inline void d_operands(int l, const uint16_t *__restrict__ Dhi_,
                                  const uint16_t *__restrict__ Dlo_, m16x4 &fh,
                                  m16x4 &fl, m16x4 &bh, m16x4 &bl) {
  const gp<const uint16_t> Dhi = (gp<const uint16_t>)Dhi_;
  const gp<const uint16_t> Dlo = (gp<const uint16_t>)Dlo_;
  const int r = l & 15, g = l >> 4;
  const bool blk = (r >> 3) == (g >> 1);
  const int a = r & 7;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = 4 * (g & 1) + q;
    const bool okf = blk && a < N1 && m < N1;
    fh[q] = okf ? (short)Dhi[a * N1 + m] : (short)0;
    fl[q] = okf ? (short)Dlo[a * N1 + m] : (short)0;
    bh[q] = okf ? (short)Dhi[m * N1 + a] : (short)0;
    bl[q] = okf ? (short)Dlo[m * N1 + a] : (short)0;
  }
}

// One element per wave.  The caller has placed the element's u (BF16,
// padded [k][j][i] order, zeros outside n1) in L.u -- with ULO, an FP32 u
// as the two-term split u = L.u + L.ul -- and holds in gq the six BF16
// factors of the lane's column (i, j) = (l % 8, l / 8) for k < 8 (zero
// outside the element).  On return L.gr holds w in [k][j][i] order.  With
// ULO each gradient contraction accumulates D_hi u_hi, D_lo u_hi and
// D_hi u_lo (the D_lo u_lo term is below the FP32 accumulation's rounding).
template <int N1, bool SPLIT, bool ULO = false, class Lds = MfmaLds>
__device__ inline void mfma_element(int l, Lds &L, const uint16_t (&gq)[6][8],
                                    m16x4 fh, m16x4 fl, m16x4 bh, m16x4 bl) {
  const int r = l & 15, g = l >> 4;
  const mf32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // ---- gradient: three contractions ----
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {
    {  // t: B from u[m][c], m = 4 (g % 2) + q, c = 32 h2 + 16 (g / 2) + r
      const int c = 32 * h2 + 16 * (g >> 1) + r, m0 = 4 * (g & 1);
      const m16x4 b = lds4_strided(&L.u[m0 * 64 + c], 64);
      mf32x4 acc = mfma(fh, b, zero);
      if (SPLIT) acc = mfma(fl, b, acc);
      if constexpr (ULO) acc = mfma(fh, lds4_strided(&L.ul[m0 * 64 + c], 64), acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) L.gt[(m0 + q) * 64 + c] = acc[q];
    }
    {  // r: A from u[rho][m], rho = 32 h2 + 16 (g / 2) + r
      const int rho = 32 * h2 + 16 * (g >> 1) + r, m0 = 4 * (g & 1);
      const m16x4 a = *reinterpret_cast<const m16x4 *>(&L.u[rho * 8 + m0]);
      mf32x4 acc = mfma(a, fh, zero);
      if (SPLIT) acc = mfma(a, fl, acc);
      if constexpr (ULO)
        acc = mfma(*reinterpret_cast<const m16x4 *>(&L.ul[rho * 8 + m0]), fh, acc);
      const int i = r & 7, rho0 = 32 * h2 + 16 * (r >> 3) + 4 * g;
#pragma unroll
      for (int q = 0; q < 4; ++q) L.gr[(rho0 + q) * 8 + i] = acc[q];
    }
    {  // s: B from u[k][m][i], k = 4 h2 + 2 (g / 2) + r / 8
      const int k = 4 * h2 + 2 * (g >> 1) + (r >> 3), i = r & 7, m0 = 4 * (g & 1);
      const m16x4 b = lds4_strided(&L.u[k * 64 + m0 * 8 + i], 8);
      mf32x4 acc = mfma(fh, b, zero);
      if (SPLIT) acc = mfma(fl, b, acc);
      if constexpr (ULO) acc = mfma(fh, lds4_strided(&L.ul[k * 64 + m0 * 8 + i], 8), acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) L.gs[k * 64 + (m0 + q) * 8 + i] = acc[q];
    }
  }
  wave_lds_sync();
  // ---- metric step on the lane's column (FP32) ----
  {
    const int i = l & 7, j = l >> 3;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int p = k * 64 + j * 8 + i;
      const float ur = L.gr[p], us = L.gs[p], ut = L.gt[p];
      const float g0 = bf16_to_f32(gq[0][k]), g1 = bf16_to_f32(gq[1][k]),
                  g2 = bf16_to_f32(gq[2][k]), g3 = bf16_to_f32(gq[3][k]),
                  g4 = bf16_to_f32(gq[4][k]), g5 = bf16_to_f32(gq[5][k]);
      L.fr[p] = f32_to_bf16(g0 * ur + g1 * us + g2 * ut);
      L.fs[p] = f32_to_bf16(g1 * ur + g3 * us + g4 * ut);
      L.ft[p] = f32_to_bf16(g2 * ur + g4 * us + g5 * ut);
    }
  }
  wave_lds_sync();
  // ---- divergence: w = D_r^T f_r + D_s^T f_s + D_t^T f_t into L.gr ----
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {  // r: A from f_r[rho][m], B = D^T blocks
    const int rho = 32 * h2 + 16 * (g >> 1) + r, m0 = 4 * (g & 1);
    const m16x4 a = *reinterpret_cast<const m16x4 *>(&L.fr[rho * 8 + m0]);
    mf32x4 acc = mfma(a, bh, zero);
    if (SPLIT) acc = mfma(a, bl, acc);
    const int i = r & 7, rho0 = 32 * h2 + 16 * (r >> 3) + 4 * g;
#pragma unroll
    for (int q = 0; q < 4; ++q) L.gr[(rho0 + q) * 8 + i] = acc[q];
  }
  wave_lds_sync();
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {  // s: A = diag(D^T), B from f_s[k][m][i]
    const int k = 4 * h2 + 2 * (g >> 1) + (r >> 3), i = r & 7, m0 = 4 * (g & 1);
    const m16x4 b = lds4_strided(&L.fs[k * 64 + m0 * 8 + i], 8);
    mf32x4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = L.gr[k * 64 + (m0 + q) * 8 + i];
    acc = mfma(bh, b, acc);
    if (SPLIT) acc = mfma(bl, b, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) L.gr[k * 64 + (m0 + q) * 8 + i] = acc[q];
  }
  wave_lds_sync();
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {  // t: A = diag(D^T), B from f_t[m][c]
    const int c = 32 * h2 + 16 * (g >> 1) + r, m0 = 4 * (g & 1);
    const m16x4 b = lds4_strided(&L.ft[m0 * 64 + c], 64);
    mf32x4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = L.gr[(m0 + q) * 64 + c];
    acc = mfma(bh, b, acc);
    if (SPLIT) acc = mfma(bl, b, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) L.gr[(m0 + q) * 64 + c] = acc[q];
  }
  wave_lds_sync();
}

// the six BF16 factors of column (i, j) of element e: the column-contiguous
// layout [E][6][64][8] at n1 = 8, [E][6][n1^3] otherwise
template <int N1>
__device__ inline void load_factors(int l, bool act, int64_t e,
                                    const uint16_t *__restrict__ G_,
                                    uint16_t (&gq)[6][8]) {
  constexpr int NP = N1 * N1, N3 = NP * N1;
  const gp<const uint16_t> G = (gp<const uint16_t>)G_;
  const int i = l & 7, j = l >> 3;
  if constexpr (N1 == 8) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (act)
        v = __builtin_nontemporal_load((gp<const u32x4>)(G + e * 6 * N3 + q * N3 + 8 * l));
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        gq[q][2 * h] = (uint16_t)(wv[h] & 0xffffu);
        gq[q][2 * h + 1] = (uint16_t)(wv[h] >> 16);
      }
    }
  } else {
    const bool col = act && i < N1 && j < N1;
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < 8; ++k)
        gq[q][k] = (col && k < N1)
                       ? G[e * 6 * N3 + q * N3 + k * NP + j * N1 + i]
                       : (uint16_t)0;
  }
}

// ---------------------------------------------------------------------------
// n1 = 9 (N = 8): the element does not fit the 8-block form.  Every
// contraction runs on 16-padded operands instead: the derivative operand is
// D (or D^T) padded to 16 x 16 with zeros, the node operand is read from the
// element's natural [k][j][i] layout in LDS with every index beyond 8
// predicated to zero, and one 16x16x16 MFMA contracts a whole length-9
// line:
//   t (over k):  C[k'][c]    = sum_m D[k'][m] u[m][c],  c = (j, i) in 6
//                tiles of 16 of the 81 columns
//   r (over i):  C[rho][i']  = sum_m u[rho][m] D[i'][m], rho = (k, j) in 6
//                tiles of 16 of the 81 rows
//   s (over j):  C[j'][i]    = sum_m D[j'][m] u[k][m][i], one MFMA per k
// (21 MFMAs per derivative term and direction set, against 6 with the
// block-diagonal 8-form; the matrix cores are far from busy either way).
// The transposed contractions use D^T the same way and accumulate w through
// the C operand (r, then s, then t).  The metric step is FP32 on the VALU,
// lane l taking the columns l and l + 64 (< 81).
// ---------------------------------------------------------------------------
constexpr int MW9 = 2;  // waves (elements) per workgroup at n1 = 9
constexpr int E9 = 729;

struct alignas(16) MfmaLds9 {
  uint16_t u[E9];
  uint16_t ul[E9];                  // low term of a split input (solver)
  float gr[E9], gs[E9], gt[E9];     // gradients; gr is reused for w
  uint16_t fr[E9], fs[E9], ft[E9];
};

// D[r][4g + q] (fwd) and D[4g + q][r] (bwd), zero outside 9 x 9
__device__ inline void d_operands9(int l, const uint16_t *__restrict__ Dhi_,
                                   const uint16_t *__restrict__ Dlo_, m16x4 &fh,
                                   m16x4 &fl, m16x4 &bh, m16x4 &bl) {
  const gp<const uint16_t> Dhi = (gp<const uint16_t>)Dhi_;
  const gp<const uint16_t> Dlo = (gp<const uint16_t>)Dlo_;
  const int r = l & 15, g = l >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = 4 * g + q;
    const bool ok = r < 9 && m < 9;
    fh[q] = ok ? (short)Dhi[r * 9 + m] : (short)0;
    fl[q] = ok ? (short)Dlo[r * 9 + m] : (short)0;
    bh[q] = ok ? (short)Dhi[m * 9 + r] : (short)0;
    bl[q] = ok ? (short)Dlo[m * 9 + r] : (short)0;
  }
}

// four BF16 values p[off(q)], q = 0..3, zero where ok(q) fails
template <class F, class O>
__device__ inline m16x4 lds4_pred(const uint16_t *p, F off, O ok) {
  m16x4 v;
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = ok(q) ? (short)p[off(q)] : (short)0;
  return v;
}

// One element per wave, u (BF16, [k][j][i], with ULO the FP32 split u =
// L.u + L.ul) in LDS; gq holds the BF16 factors of the lane's columns l and
// l + 64 for k = 0..8.  On return L.gr holds w in [k][j][i] order.
template <bool SPLIT, bool ULO>
__device__ inline void mfma_element9(int l, MfmaLds9 &L, const uint16_t (&gq)[2][6][9],
                                     m16x4 fh, m16x4 fl, m16x4 bh, m16x4 bl) {
  const int r = l & 15, g = l >> 4;
  const mf32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // ---- gradient ----
#pragma unroll
  for (int t = 0; t < 6; ++t) {  // t: columns c = 16 t + r
    const int c = 16 * t + r;
    auto off = [&](int q) { return (4 * g + q) * 81 + c; };
    auto ok = [&](int q) { return 4 * g + q < 9 && c < 81; };
    const m16x4 b = lds4_pred(L.u, off, ok);
    mf32x4 acc = mfma(fh, b, zero);
    if (SPLIT) acc = mfma(fl, b, acc);
    if constexpr (ULO) acc = mfma(fh, lds4_pred(L.ul, off, ok), acc);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * g + q < 9 && c < 81) L.gt[(4 * g + q) * 81 + c] = acc[q];
  }
#pragma unroll
  for (int t = 0; t < 6; ++t) {  // r: rows rho = 16 t + r of u[rho][m]
    const int rho = 16 * t + r;
    auto off = [&](int q) { return rho * 9 + 4 * g + q; };
    auto ok = [&](int q) { return rho < 81 && 4 * g + q < 9; };
    const m16x4 a = lds4_pred(L.u, off, ok);
    mf32x4 acc = mfma(a, fh, zero);
    if (SPLIT) acc = mfma(a, fl, acc);
    if constexpr (ULO) acc = mfma(lds4_pred(L.ul, off, ok), fh, acc);
    // C[rho'][i'] with rho' = 16 t + 4 g + q, i' = r
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = 16 * t + 4 * g + q;
      if (rr < 81 && r < 9) L.gr[rr * 9 + r] = acc[q];
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {  // s: B[m][i] = u[k][m][i]
    auto off = [&](int q) { return k * 81 + (4 * g + q) * 9 + r; };
    auto ok = [&](int q) { return 4 * g + q < 9 && r < 9; };
    const m16x4 b = lds4_pred(L.u, off, ok);
    mf32x4 acc = mfma(fh, b, zero);
    if (SPLIT) acc = mfma(fl, b, acc);
    if constexpr (ULO) acc = mfma(fh, lds4_pred(L.ul, off, ok), acc);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * g + q < 9 && r < 9) L.gs[k * 81 + (4 * g + q) * 9 + r] = acc[q];
  }
  wave_lds_sync();
  // ---- metric step on the lane's columns (FP32) ----
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = l + 64 * h;
    if (c < 81) {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int p = k * 81 + c;
        const float ur = L.gr[p], us = L.gs[p], ut = L.gt[p];
        const float g0 = bf16_to_f32(gq[h][0][k]), g1 = bf16_to_f32(gq[h][1][k]),
                    g2 = bf16_to_f32(gq[h][2][k]), g3 = bf16_to_f32(gq[h][3][k]),
                    g4 = bf16_to_f32(gq[h][4][k]), g5 = bf16_to_f32(gq[h][5][k]);
        L.fr[p] = f32_to_bf16(g0 * ur + g1 * us + g2 * ut);
        L.fs[p] = f32_to_bf16(g1 * ur + g3 * us + g4 * ut);
        L.ft[p] = f32_to_bf16(g2 * ur + g4 * us + g5 * ut);
      }
    }
  }
  wave_lds_sync();
  // ---- divergence into L.gr ----
#pragma unroll
  for (int t = 0; t < 6; ++t) {  // r: A = f_r[rho][m], B[m][i] = D[m][i]
    const int rho = 16 * t + r;
    auto off = [&](int q) { return rho * 9 + 4 * g + q; };
    auto ok = [&](int q) { return rho < 81 && 4 * g + q < 9; };
    const m16x4 a = lds4_pred(L.fr, off, ok);
    mf32x4 acc = mfma(a, bh, zero);
    if (SPLIT) acc = mfma(a, bl, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = 16 * t + 4 * g + q;
      if (rr < 81 && r < 9) L.gr[rr * 9 + r] = acc[q];
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 9; ++k) {  // s: A[j][m] = D[m][j], B[m][i] = f_s[k][m][i]
    auto off = [&](int q) { return k * 81 + (4 * g + q) * 9 + r; };
    auto ok = [&](int q) { return 4 * g + q < 9 && r < 9; };
    const m16x4 b = lds4_pred(L.fs, off, ok);
    mf32x4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = ok(q) ? L.gr[off(q)] : 0.f;
    acc = mfma(bh, b, acc);
    if (SPLIT) acc = mfma(bl, b, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (ok(q)) L.gr[off(q)] = acc[q];
  }
  wave_lds_sync();
#pragma unroll
  for (int t = 0; t < 6; ++t) {  // t: A[k][m] = D[m][k], B[m][c] = f_t[m][c]
    const int c = 16 * t + r;
    auto off = [&](int q) { return (4 * g + q) * 81 + c; };
    auto ok = [&](int q) { return 4 * g + q < 9 && c < 81; };
    const m16x4 b = lds4_pred(L.ft, off, ok);
    mf32x4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = ok(q) ? L.gr[off(q)] : 0.f;
    acc = mfma(bh, b, acc);
    if (SPLIT) acc = mfma(bl, b, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (ok(q)) L.gr[off(q)] = acc[q];
  }
  wave_lds_sync();
}

// the BF16 factors of columns l and l + 64 of element e ([E][6][729])
__device__ inline void load_factors9(int l, bool act, int64_t e,
                                     const uint16_t *__restrict__ G_,
                                     uint16_t (&gq)[2][6][9]) {
  const gp<const uint16_t> G = (gp<const uint16_t>)G_;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = l + 64 * h;
    const bool col = act && c < 81;
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
      for (int k = 0; k < 9; ++k)
        gq[h][q][k] = col ? G[e * 6 * E9 + q * E9 + k * 81 + c] : (uint16_t)0;
  }
}

template <bool SPLIT>
__global__ void __launch_bounds__(64 * MW9)
    k_ax_mfma9(int64_t E, const uint16_t *__restrict__ Dhi,
               const uint16_t *__restrict__ Dlo, const uint16_t *__restrict__ G,
               const uint16_t *__restrict__ H, const uint16_t *__restrict__ u,
               float *__restrict__ w) {
  __shared__ MfmaLds9 lds[MW9];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * MW9 + wv;
  const bool act = e < E;
  MfmaLds9 &L = lds[wv];
  m16x4 fh, fl, bh, bl;
  d_operands9(l, Dhi, Dlo, fh, fl, bh, bl);
  uint16_t gq[2][6][9];
  load_factors9(l, act, e, G, gq);
  for (int p = l; p < E9; p += 64) L.u[p] = act ? u[e * E9 + p] : (uint16_t)0;
  wave_lds_sync();
  mfma_element9<SPLIT, false>(l, L, gq, fh, fl, bh, bl);
  if (!act) return;  // no barrier follows
  for (int p = l; p < E9; p += 64) {
    float v = L.gr[p];
    if (H != nullptr) v += bf16_to_f32(H[e * E9 + p]) * bf16_to_f32(L.u[p]);
    w[e * E9 + p] = v;
  }
}

// ---------------------------------------------------------------------------
// standalone operator: BF16 E-vector in, FP32 E-vector out
// ---------------------------------------------------------------------------
template <int N1, bool SPLIT>
__global__ void __launch_bounds__(64 * MW)
    k_ax_mfma(int64_t E, const uint16_t *__restrict__ Dhi,
              const uint16_t *__restrict__ Dlo, const uint16_t *__restrict__ G,
              const uint16_t *__restrict__ H, const uint16_t *__restrict__ u,
              float *__restrict__ w) {
  constexpr int NP = N1 * N1, N3 = NP * N1;
  __shared__ MfmaLds lds[MW];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * MW + wv;
  const bool act = e < E;
  MfmaLds &L = lds[wv];
  m16x4 fh, fl, bh, bl;
  d_operands<N1>(l, Dhi, Dlo, fh, fl, bh, bl);
  uint16_t gq[6][8];
  load_factors<N1>(l, act, e, G, gq);
  if constexpr (N1 == 8) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (act) v = *reinterpret_cast<const u32x4 *>(u + e * N3 + 8 * l);
    *reinterpret_cast<u32x4 *>(&L.u[8 * l]) = v;
  } else {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int p = l + 64 * t, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
      L.u[p] = (act && i < N1 && j < N1 && k < N1) ? u[e * N3 + k * NP + j * N1 + i]
                                                   : (uint16_t)0;
    }
  }
  wave_lds_sync();
  mfma_element<N1, SPLIT>(l, L, gq, fh, fl, bh, bl);
  if (!act) return;  // no barrier follows
  if constexpr (N1 == 8) {
    const float *src = &L.gr[8 * l];
    float hv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (H != nullptr) {  // uniform
      const u32x4 v =
          __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(H + e * N3 + 8 * l));
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        hv[2 * h] = bf16_to_f32((uint16_t)(wv[h] & 0xffffu)) * bf16_to_f32(L.u[8 * l + 2 * h]);
        hv[2 * h + 1] =
            bf16_to_f32((uint16_t)(wv[h] >> 16)) * bf16_to_f32(L.u[8 * l + 2 * h + 1]);
      }
    }
#pragma unroll
    for (int h = 0; h < 8; ++h)
      __builtin_nontemporal_store(src[h] + hv[h], w + e * N3 + 8 * l + h);
  } else {
    for (int p = l; p < N3; p += 64) {
      const int i = p % N1, j = (p / N1) % N1, k = p / NP;
      const int q = k * 64 + j * 8 + i;
      float v = L.gr[q];
      if (H != nullptr) v += bf16_to_f32(H[e * N3 + p]) * bf16_to_f32(L.u[q]);
      w[e * N3 + p] = v;
    }
  }
}

template <bool SPLIT>
static void launch_ax_mfma_s(int N, int64_t E, const uint16_t *Dhi,
                             const uint16_t *Dlo, const uint16_t *G,
                             const uint16_t *H, const uint16_t *u, float *w,
                             hipStream_t s) {
  const int64_t blocks = (E + MW - 1) / MW;
  if (blocks == 0) return;
  const dim3 grid((unsigned)blocks), block(64 * MW);
  switch (N) {
#define SEM_AXM(NN)                                                          \
  case NN:                                                                   \
    hipLaunchKernelGGL((k_ax_mfma<NN + 1, SPLIT>), grid, block, 0, s, E, Dhi, \
                       Dlo, G, H, u, w);                                     \
    break;
    SEM_AXM(1)
    SEM_AXM(2)
    SEM_AXM(3)
    SEM_AXM(4)
    SEM_AXM(5)
    SEM_AXM(6)
    SEM_AXM(7)
#undef SEM_AXM
    case 8:
      hipLaunchKernelGGL((k_ax_mfma9<SPLIT>), dim3((unsigned)((E + MW9 - 1) / MW9)),
                         dim3(64 * MW9), 0, s, E, Dhi, Dlo, G, H, u, w);
      break;
    default:
      fail(SEM_ERR_ARG, "sem_ax: the matrix-core operator needs N in 1..8");
  }
}

void launch_ax_mfma(int N, bool split, int64_t E, const uint16_t *Dhi,
                    const uint16_t *Dlo, const uint16_t *G, const uint16_t *H,
                    const uint16_t *u, float *w, hipStream_t s) {
  if (split)
    launch_ax_mfma_s<true>(N, E, Dhi, Dlo, G, H, u, w, s);
  else
    launch_ax_mfma_s<false>(N, E, Dhi, Dlo, G, H, u, w, s);
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// batched operator inside the solvers: FP32 unique-node input gathered
// through the box numbering and split into two BF16 terms (u_hi = bf16(u),
// u_lo = bf16(u - u_hi)), FP32 E-vector output; items are tiles of a single
// order (n1 = N1s), MW elements per workgroup pass.  Rounding the input to
// BF16 alone leaves an input error that refinement cannot remove at scale:
// A (I + Delta) p with |Delta| ~ 2^-9 amplifies rough components by the
// operator's spread of eigenvalues, and the refinement's contraction grew
// with the mesh (0.36 per step at 32^3 elements, N = 7).
// ---------------------------------------------------------------------------
// want_edot: also store every element's energy p_e^T w_e in FP64 (the terms
// of (p, A p) for the solvers), each lane's column of the FP32 input p times
// the stored w in ascending k, then the lanes by a fixed butterfly
// One element of the solvers' operator (gathered FP32 input p, split into
// two BF16 terms; FP32 output; with edot non-null the element energy).
// Every wave of the workgroup calls it (act = false: no loads or stores),
// since the element routine synchronises the workgroup.
template <int N1, bool SPLIT>
__device__ inline void solve_elem_mfma(int l, MfmaLdsSplit &L, int64_t e, bool act,
                                       const Box &box, gp<const float> u, gp<float> w,
                                       const uint16_t *G, gp<const uint16_t> H,
                                       m16x4 fh, m16x4 fl, m16x4 bh, m16x4 bl,
                                       gp<double> edot) {
  constexpr int NP = N1 * N1, N3 = NP * N1;
  uint16_t gq[6][8];
  load_factors<N1>(l, act, e, G, gq);
  ElemXYZ c3 = {0u, 0u, 0u};
  if (act) c3 = box_elem(box, (uint32_t)e);
  float pv[8];  // the lane's column (i, j) = (l % 8, l / 8) of p, k = t
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int p = l + 64 * t, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const bool in = act && i < N1 && j < N1 && k < N1;
    const float v = in ? u[box_node(box, c3, i, j, k)] : 0.f;
    pv[t] = v;
    const uint16_t hi = f32_to_bf16(v);
    L.u[p] = hi;
    L.ul[p] = f32_to_bf16(v - bf16_to_f32(hi));
  }
  wave_lds_sync();
  mfma_element<N1, SPLIT, true, MfmaLdsSplit>(l, L, gq, fh, fl, bh, bl);
  // w at node (i, j, k) of the element, as stored (mass term added)
  auto wval = [&](int i, int j, int k) {
    const int q = k * 64 + j * 8 + i;
    float v = L.gr[q];
    if (H != nullptr)
      v += bf16_to_f32(H[e * N3 + k * NP + j * N1 + i]) *
           (bf16_to_f32(L.u[q]) + bf16_to_f32(L.ul[q]));
    return v;
  };
  if (act) {
    for (int p = l; p < N3; p += 64) w[e * N3 + p] = wval(p % N1, (p / N1) % N1, p / NP);
  }
  if (edot != nullptr) {  // uniform
    const int i = l & 7, j = l >> 3;
    double cd = 0.0;
    if (i < N1 && j < N1) {
#pragma unroll
      for (int t = 0; t < N1; ++t) cd += (double)pv[t] * (double)wval(i, j, t);
    }
    cd = wave_sum(cd);
    if (act && l == 0) edot[e] = cd;
  }
}

// want_edot: also store every element's energy p_e^T w_e in FP64 (the terms
// of (p, A p) for the solvers), each lane's column of the FP32 input p times
// the stored w in ascending k, then the lanes by a fixed butterfly
template <int N1, bool SPLIT>
__global__ void __launch_bounds__(64 * MW)
    k_bax_mfma(const BatchSolve *__restrict__ sds, const CgState *__restrict__ st,
               const AxItem *__restrict__ items, int nitems, int epb, int src,
               int dst, int skip_done, int want_edot) {
  __shared__ MfmaLdsSplit lds[MW];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  MfmaLdsSplit &L = lds[wv];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const AxItem it = items[q];
    if (skip_done && st[it.solve].done != 0) continue;  // uniform per block
    const BatchSolve &sd = sds[it.solve];
    m16x4 fh, fl, bh, bl;
    d_operands<N1>(l, (const uint16_t *)sd.D16hi, (const uint16_t *)sd.D16lo, fh,
                   fl, bh, bl);
    for (int e0 = 0; e0 < epb; e0 += MW) {  // uniform per block
      const int64_t e = it.elem0 + e0 + wv;
      // global pointers (their address space is not known from the descriptor)
      solve_elem_mfma<N1, SPLIT>(
          l, L, e, e0 + wv < epb && e < sd.E, sd.box, (gp<const float>)sd.v32[src],
          (gp<float>)sd.v32[dst], (const uint16_t *)sd.G16, (gp<const uint16_t>)sd.H16,
          fh, fl, bh, bl, want_edot ? (gp<double>)sd.edot : nullptr);
      wave_lds_sync();  // L is reused by the next element
    }
  }
}

// The same operator for a single solve, every argument passed in (no work
// item or descriptor to fetch first), one element per wave; a finished
// solve's workgroups return at once.
template <int N1, bool SPLIT>
__global__ void __launch_bounds__(64 * MW)
    k_ax_mfma_solve(int64_t E, const uint16_t *__restrict__ Dhi,
                    const uint16_t *__restrict__ Dlo, const uint16_t *__restrict__ G,
                    const uint16_t *__restrict__ H, const float *__restrict__ u,
                    float *__restrict__ w, Box box, const int32_t *__restrict__ stop,
                    double *__restrict__ edot) {
  __shared__ MfmaLdsSplit lds[MW];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (stop != nullptr && *stop != 0) return;  // uniform: the solve is done
  m16x4 fh, fl, bh, bl;
  d_operands<N1>(l, Dhi, Dlo, fh, fl, bh, bl);
  const int64_t e = (int64_t)blockIdx.x * MW + wv;
  solve_elem_mfma<N1, SPLIT>(l, lds[wv], e, e < E, box, (gp<const float>)u, (gp<float>)w,
                             G, (gp<const uint16_t>)H, fh, fl, bh, bl,
                             (gp<double>)edot);
}

// one element of the solvers' operator at n1 = 9 (as solve_elem_mfma)
template <bool SPLIT>
__device__ inline void solve_elem_mfma9(int l, MfmaLds9 &L, int64_t e, bool act,
                                        const Box &box, gp<const float> u, gp<float> w,
                                        const uint16_t *G, gp<const uint16_t> H,
                                        m16x4 fh, m16x4 fl, m16x4 bh, m16x4 bl,
                                        gp<double> edot) {
  uint16_t gq[2][6][9];
  load_factors9(l, act, e, G, gq);
  ElemXYZ c3 = {0u, 0u, 0u};
  if (act) c3 = box_elem(box, (uint32_t)e);
  constexpr int T9 = (E9 + 63) / 64;
  float pv[T9];  // p at the lane's nodes p = l + 64 t
#pragma unroll
  for (int t = 0; t < T9; ++t) {
    const int p = l + 64 * t;
    if (p < E9) {
      const int i = p % 9, j = (p / 9) % 9, k = p / 81;
      const float v = act ? u[box_node(box, c3, i, j, k)] : 0.f;
      pv[t] = v;
      const uint16_t hi = f32_to_bf16(v);
      L.u[p] = hi;
      L.ul[p] = f32_to_bf16(v - bf16_to_f32(hi));
    } else {
      pv[t] = 0.f;
    }
  }
  wave_lds_sync();
  mfma_element9<SPLIT, true>(l, L, gq, fh, fl, bh, bl);
  auto wval = [&](int p) {  // w at node p, as stored (mass term added)
    float v = L.gr[p];
    if (H != nullptr)
      v += bf16_to_f32(H[e * E9 + p]) * (bf16_to_f32(L.u[p]) + bf16_to_f32(L.ul[p]));
    return v;
  };
  if (act) {
    for (int p = l; p < E9; p += 64) w[e * E9 + p] = wval(p);
  }
  if (edot != nullptr) {  // uniform; each lane's nodes in ascending t, then the lanes
    double cd = 0.0;
#pragma unroll
    for (int t = 0; t < T9; ++t)
      if (l + 64 * t < E9) cd += (double)pv[t] * (double)wval(l + 64 * t);
    cd = wave_sum(cd);
    if (act && l == 0) edot[e] = cd;
  }
}

// the batched solver operator at n1 = 9: as k_bax_mfma, MW9 elements per
// workgroup pass
template <bool SPLIT>
__global__ void __launch_bounds__(64 * MW9)
    k_bax_mfma9(const BatchSolve *__restrict__ sds, const CgState *__restrict__ st,
                const AxItem *__restrict__ items, int nitems, int epb, int src,
                int dst, int skip_done, int want_edot) {
  __shared__ MfmaLds9 lds[MW9];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  MfmaLds9 &L = lds[wv];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const AxItem it = items[q];
    if (skip_done && st[it.solve].done != 0) continue;  // uniform per block
    const BatchSolve &sd = sds[it.solve];
    m16x4 fh, fl, bh, bl;
    d_operands9(l, (const uint16_t *)sd.D16hi, (const uint16_t *)sd.D16lo, fh, fl,
                bh, bl);
    for (int e0 = 0; e0 < epb; e0 += MW9) {  // uniform per block
      const int64_t e = it.elem0 + e0 + wv;
      solve_elem_mfma9<SPLIT>(
          l, L, e, e0 + wv < epb && e < sd.E, sd.box, (gp<const float>)sd.v32[src],
          (gp<float>)sd.v32[dst], (const uint16_t *)sd.G16, (gp<const uint16_t>)sd.H16,
          fh, fl, bh, bl, want_edot ? (gp<double>)sd.edot : nullptr);
      wave_lds_sync();  // L is reused by the next element
    }
  }
}

// the single-solve operator at n1 = 9 (as k_ax_mfma_solve)
template <bool SPLIT>
__global__ void __launch_bounds__(64 * MW9)
    k_ax_mfma_solve9(int64_t E, const uint16_t *__restrict__ Dhi,
                     const uint16_t *__restrict__ Dlo, const uint16_t *__restrict__ G,
                     const uint16_t *__restrict__ H, const float *__restrict__ u,
                     float *__restrict__ w, Box box, const int32_t *__restrict__ stop,
                     double *__restrict__ edot) {
  __shared__ MfmaLds9 lds[MW9];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (stop != nullptr && *stop != 0) return;  // uniform: the solve is done
  m16x4 fh, fl, bh, bl;
  d_operands9(l, Dhi, Dlo, fh, fl, bh, bl);
  const int64_t e = (int64_t)blockIdx.x * MW9 + wv;
  solve_elem_mfma9<SPLIT>(l, lds[wv], e, e < E, box, (gp<const float>)u, (gp<float>)w, G,
                          (gp<const uint16_t>)H, fh, fl, bh, bl, (gp<double>)edot);
}

void launch_ax_mfma_solve(int N, bool split, int64_t E, const uint16_t *Dhi,
                          const uint16_t *Dlo, const uint16_t *G, const uint16_t *H,
                          const float *u, float *w, const Box &box, const int32_t *stop,
                          double *edot, hipStream_t s) {
  if (E <= 0) return;
  const int n1 = N + 1;
  if (n1 == 9) {
    const dim3 g((unsigned)((E + MW9 - 1) / MW9)), b(64 * MW9);
    if (split)
      hipLaunchKernelGGL((k_ax_mfma_solve9<true>), g, b, 0, s, E, Dhi, Dlo, G, H, u, w,
                         box, stop, edot);
    else
      hipLaunchKernelGGL((k_ax_mfma_solve9<false>), g, b, 0, s, E, Dhi, Dlo, G, H, u, w,
                         box, stop, edot);
    SEM_HIP(hipGetLastError());
    return;
  }
  const dim3 g((unsigned)((E + MW - 1) / MW)), b(64 * MW);
  switch (n1) {
#define SEM_AXMS(NN)                                                                  \
  case NN:                                                                            \
    if (split)                                                                        \
      hipLaunchKernelGGL((k_ax_mfma_solve<NN, true>), g, b, 0, s, E, Dhi, Dlo, G, H,  \
                         u, w, box, stop, edot);                                      \
    else                                                                              \
      hipLaunchKernelGGL((k_ax_mfma_solve<NN, false>), g, b, 0, s, E, Dhi, Dlo, G, H, \
                         u, w, box, stop, edot);                                      \
    break;
    SEM_AXMS(2)
    SEM_AXMS(3)
    SEM_AXMS(4)
    SEM_AXMS(5)
    SEM_AXMS(6)
    SEM_AXMS(7)
    SEM_AXMS(8)
#undef SEM_AXMS
    default:
      fail(SEM_ERR_ARG, "solve: the matrix-core operator needs N in 1..8");
  }
  SEM_HIP(hipGetLastError());
}

void launch_bax_mfma(int n1, bool split, const BatchSolve *sds, const CgState *st,
                     const AxItem *items, int nitems, int epb, int grid, int src,
                     int dst, int skip_done, bool edot, hipStream_t s) {
  const int want_edot = edot ? 1 : 0;
  if (nitems <= 0) return;
  const dim3 g((unsigned)grid), b(64 * MW);
  switch (n1) {
#define SEM_BAXM(NN)                                                            \
  case NN:                                                                      \
    if (split)                                                                  \
      hipLaunchKernelGGL((k_bax_mfma<NN, true>), g, b, 0, s, sds, st, items,    \
                         nitems, epb, src, dst, skip_done, want_edot);          \
    else                                                                        \
      hipLaunchKernelGGL((k_bax_mfma<NN, false>), g, b, 0, s, sds, st, items,   \
                         nitems, epb, src, dst, skip_done, want_edot);          \
    break;
    SEM_BAXM(2)
    SEM_BAXM(3)
    SEM_BAXM(4)
    SEM_BAXM(5)
    SEM_BAXM(6)
    SEM_BAXM(7)
    SEM_BAXM(8)
#undef SEM_BAXM
    case 9: {
      const dim3 b9(64 * MW9);
      if (split)
        hipLaunchKernelGGL((k_bax_mfma9<true>), g, b9, 0, s, sds, st, items, nitems,
                           epb, src, dst, skip_done, want_edot);
      else
        hipLaunchKernelGGL((k_bax_mfma9<false>), g, b9, 0, s, sds, st, items, nitems,
                           epb, src, dst, skip_done, want_edot);
      break;
    }
    default:
      fail(SEM_ERR_ARG, "batched operator: the matrix-core operator needs N in 1..8");
  }
  SEM_HIP(hipGetLastError());
}

}  // namespace sem
