// Preconditioned conjugate gradients for the assembled SEM system (paper
// section 4.2.2: the system is solved by PCG, whose dominant cost is the
// operator application), FP64 iterative refinement around an FP32 /
// BF16-operator inner PCG, and batches of independent solves of uneven size
// and order.
//
// Everything runs on batches: a single solve is a batch of one.  Vectors
// live on unique (global) nodes; the operator is applied as
//   w_G = mask o Q^T A_L Q p_G
// with Q fused into the operator kernel (gather through the closed-form
// numbering).  p vanishes on Dirichlet nodes, so (p, w_G) = sum_e p_e^T w_e:
// the operator stores the element energies and the assembled w_G is never
// stored -- the r update sums the copies of each node itself (Q^T + mask).
// One CG iteration of the whole batch is five launches of persistent
// kernels that walk work lists of (solve, element tile) or (solve, node
// chunk) items:
//   operator + element energies -> alpha -> assembly + r update +
//   z = dinv r + dots -> beta / convergence -> x and p update.
// (The matrix-core operator has no energy output: with it the iteration
// keeps a separate assembly with the (p, w) dot, and r, z and the dots in
// one more pass.)
// Scalars stay on the device, one CgState per solve; kernels skip items of
// solves whose flag says they finished, so a captured HIP graph of K
// iterations is replayed between host polls without changing any iterate.
// Every reduction has a fixed partition (one partial per work item) and a
// fixed summation order: results are bit-reproducible, and a solve gives the
// same bits alone or inside any batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <type_traits>
#include <sstream>
#include <string>

#include "assemble.h"
#include "common.h"
#include "sem_internal.h"

namespace sem {

constexpr int RT = 256;           // threads of the vector kernels
static_assert(VCH % RT == 0, "chunk must be a multiple of the block");

// --------------------------------------------------------------------------
// per-solve sums of the per-item partials
// --------------------------------------------------------------------------
// Thread t of a workgroup adds part[a * stride + q] for q = begin + t,
// begin + t + RT, ... < end into acc[a], in that order (the same order as a
// plain loop, so the sums are unchanged); the loads are issued PF at a time,
// so that the single workgroup of a scalar kernel does not wait for one load
// after the other.  The last batch is predicated: an absent entry adds +0.0,
// which leaves a sum that starts at +0.0 unchanged bit for bit.
template <int NA>
__device__ inline void strided_sums(const double *__restrict__ part, int stride,
                                    int begin, int end, double (&acc)[NA]) {
  // 11.4M unique nodes make 11124 chunks: 44 partials per thread, all in
  // flight at once
  constexpr int PF = NA >= 3 ? 24 : 48;
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = 0.0;
  for (int q = begin + (int)threadIdx.x; q < end; q += PF * RT) {
    double v[NA][PF];
#pragma unroll
    for (int u = 0; u < PF; ++u)
#pragma unroll
      for (int a = 0; a < NA; ++a)
        v[a][u] = q + u * RT < end ? part[a * stride + q + u * RT] : 0.0;
#pragma unroll
    for (int u = 0; u < PF; ++u)
#pragma unroll
      for (int a = 0; a < NA; ++a) acc[a] += v[a][u];
  }
}


// --------------------------------------------------------------------------
// vector kernels (persistent over VecItem lists)
// --------------------------------------------------------------------------
// the solve's vectors as global pointers (see gp)
template <class TV> __device__ inline gp<TV> vec(const BatchSolve &s, int v) {
  return (gp<TV>)(sizeof(TV) == 8 ? s.v64[v] : s.v32[v]);
}
template <class TD> __device__ inline gp<const TD> dinv_of(const BatchSolve &s,
                                                           int jac) {
  if constexpr (sizeof(TD) == 8)
    return (gp<const TD>)(jac ? s.dinv64 : s.one64);
  else
    return (gp<const TD>)(jac ? s.dinv32 : s.one32);
}

// w = mask o Q^T wL (sum of copies in ascending local index, from +0: the
// summation order of sem_gs); optional partial (p, w) per item
template <class TV, bool DOT, bool PER>
__global__ void __launch_bounds__(RT)
    k_bassemble(const BatchSolve *__restrict__ sds, const CgState *__restrict__ st,
                const VecItem *__restrict__ items, int nitems,
                double *__restrict__ part, int skip_done) {
  __shared__ double sm[RT / 64];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (skip_done && st[it.solve].done != 0) continue;
    const BatchSolve &sd = sds[it.solve];
    const Box &bx = sd.box;
    gp<const TV> wL = vec<TV>(sd, VWL);
    gp<TV> wG = vec<TV>(sd, VW);
    gp<const TV> p = vec<TV>(sd, VP);
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    double acc = 0.0;
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT) {
      const NodeCopies nc = node_copies<PER>(bx, (uint32_t)g);
      TV s = TV(0);
      if (!nc.masked) {
        // all (up to 8) copies loaded at once, predicated on existence, then
        // summed in ascending local index (z, y, x copy order); an absent
        // copy adds +0.0, which leaves the sum unchanged bit for bit (the
        // sum starts at +0.0 and so is never -0.0).  Loading them one after
        // another cost 30 % more time; four nodes per thread at once, 30 %
        // more again (registers)
        TV v[8];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const bool ok = a < nc.z.cnt && b < nc.y.cnt && c < nc.x.cnt;
              const int64_t lid = ok ? copy_lid(bx, nc, a, b, c) : 0;
              v[4 * a + 2 * b + c] = ok ? wL[lid] : TV(0);
            }
        s = sum_copies(PER ? bx.order : 0, v);
      }
      wG[g] = s;
      if (DOT) acc += (double)p[g] * (double)s;
    }
    if (DOT) {
      const double t = block_sum<RT>(acc, sm);
      if (threadIdx.x == 0) part[q] = t;
    }
  }
}

// alpha_s = rz_s / (p, A p)_s with (p, A p) the sum of the solve's element
// energies in element order (strided over the workgroup's threads, then the
// fixed workgroup sum), one workgroup of AT threads per solve
constexpr int AT = 1024;
__global__ void __launch_bounds__(AT)
    k_balpha_e(const BatchSolve *__restrict__ sds, CgState *st) {
  __shared__ double sm[AT / 64];
  const int s = blockIdx.x;
  if (threadIdx.x == 0) st[s].xupd = 0;  // no x update from an earlier step
  if (st[s].done != 0) return;
  gp<const double> ed = (gp<const double>)sds[s].edot;
  const int64_t E = sds[s].E;
  constexpr int PF = 32;  // 32768 elements: every energy loaded at once
  double acc = 0.0;
  int64_t q = threadIdx.x;
  for (; q + (PF - 1) * AT < E; q += PF * AT) {
    double v[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) v[u] = ed[q + u * AT];
#pragma unroll
    for (int u = 0; u < PF; ++u) acc += v[u];
  }
  for (; q < E; q += AT) acc += ed[q];
  const double pw = block_sum<AT>(acc, sm);
  if (threadIdx.x == 0) {
    st[s].pw = pw;
    if (!(pw > 0.0) || !isfinite(pw))
      st[s].done = 2;
    else
      st[s].alpha = st[s].rz / pw;
  }
}

// r -= alpha w_G with w_G = mask o Q^T w_L formed here (the copies of each
// node summed from +0.0 in ascending local index, as the assembly and
// sem_gs sum them), z = dinv r; partials (r, z), (r, r).  FCG (flexible CG
// with the learned correction, which the next kernel adds to z): partials
// (r, z), (z, w_G), (r, r).  xr_asm_chunk updates the chunk [start, start +
// VCH) of unique nodes; k_bupdate_xr_asm walks the work items of a batch,
// k_xr_asm_1 the chunks of a single solve.
// a load / store with the streaming (non-temporal) hint when NT
template <bool NT, class P> __device__ inline auto ld_h(P p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, class T, class P> __device__ inline void st_h(T v, P p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <class TV, class TD, bool FCG, bool PER, bool W64, bool NT>
__device__ __forceinline__ void xr_asm_chunk(const Box &bx, gp<const TV> wL, gp<TV> r,
                                             gp<TV> z, gp<const TD> dinv, TV alpha,
                                             int64_t start, int64_t nG, int q, int nitems,
                                             double *__restrict__ part, double *sm) {
  const int64_t end = min(start + (int64_t)VCH, nG);
  // w_G at the node with coordinates pc (32-bit local indices unless W64:
  // some local index of the batch needs more)
  using IT = typename std::conditional<W64, int64_t, uint32_t>::type;
  auto assembled = [&](const Coord3 &pc) { return assemble_node<TV, PER, IT>(bx, wL, pc); };
  double rz = 0.0, rr = 0.0, zw = 0.0;
  constexpr int K = VCH / RT;
  const int64_t g0 = start + threadIdx.x;
  if (g0 + (K - 1) * RT < end) {
    // a whole chunk: every load of the thread's K nodes before any store
    // (the compiler cannot know that w_L, r, z and dinv do not overlap).
    // NT (a working set beyond the last-level cache): r and dinv stream
    // non-temporally (next read an iteration later), z is stored normally
    // for the x / p update right after: FP64 100 -> 87 us at 32^3, N = 7
    TV sw[K], rv[K];
    TD dv[K];
    // the thread's nodes are RT apart: their coordinates advance by carries
    Coord3 pc = box_coord(bx, (uint32_t)g0);
    const Coord3 step = box_coord(bx, (uint32_t)RT);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      sw[k] = assembled(pc);
      rv[k] = ld_h<NT>(r + g0 + k * RT);
      dv[k] = ld_h<NT>(dinv + g0 + k * RT);
      box_advance(bx, step, pc);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const TV rn = rv[k] - alpha * sw[k];
      st_h<NT>(rn, r + g0 + k * RT);
      const TV zn = (TV)(dv[k] * rn);
      z[g0 + k * RT] = zn;
      rz += (double)rn * (double)zn;
      rr += (double)rn * (double)rn;
      if constexpr (FCG) zw += (double)zn * (double)sw[k];
    }
  } else {
    for (int64_t g = g0; g < end; g += RT) {
      const TV sg = assembled(box_coord(bx, (uint32_t)g));
      const TV rn = r[g] - alpha * sg;
      r[g] = rn;
      const TV zn = (TV)(dinv[g] * rn);
      z[g] = zn;
      rz += (double)rn * (double)zn;
      rr += (double)rn * (double)rn;
      if constexpr (FCG) zw += (double)zn * (double)sg;
    }
  }
  const double trz = block_sum<RT>(rz, sm);
  const double trr = block_sum<RT>(rr, sm);
  const double tzw = FCG ? block_sum<RT>(zw, sm) : 0.0;
  if (threadIdx.x == 0) {
    part[q] = trz;
    if constexpr (FCG) {
      part[nitems + q] = tzw;
      part[2 * nitems + q] = trr;
    } else {
      part[nitems + q] = trr;
    }
  }
}

template <class TV, class TD, bool FCG, bool PER, bool W64, bool NT>
__global__ void __launch_bounds__(RT)
    k_bupdate_xr_asm(const BatchSolve *__restrict__ sds,
                     const CgState *__restrict__ st,
                     const VecItem *__restrict__ items, int nitems,
                     double *__restrict__ part, int jac) {
  __shared__ double sm[RT / 64];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (st[it.solve].done != 0) continue;
    const BatchSolve &sd = sds[it.solve];
    xr_asm_chunk<TV, TD, FCG, PER, W64, NT>(
        sd.box, vec<TV>(sd, VWL), vec<TV>(sd, VR), vec<TV>(sd, VZ), dinv_of<TD>(sd, jac),
        (TV)st[it.solve].alpha, it.start, sd.nG, q, nitems, part, sm);
  }
}

// The vectors of a single solve, passed to the kernels of the single-solve
// iteration by value: a workgroup then reads only the solve's state before
// its data loads, where the batched kernels first fetch a work item and the
// solve's descriptor (a chain of dependent loads in front of every chunk)
template <class TV, class TD> struct Vecs1 {
  Box box;
  int64_t nG;
  const TV *wL;
  TV *r, *z, *p, *x;
  const TD *dinv;
};

template <class TV, class TD, bool FCG, bool PER, bool W64, bool NT>
__global__ void __launch_bounds__(RT)
    k_xr_asm_1(Vecs1<TV, TD> a, const CgState *__restrict__ st, int nitems,
               double *__restrict__ part) {
  __shared__ double sm[RT / 64];
  if (st->done != 0) return;
  const int q = blockIdx.x;
  xr_asm_chunk<TV, TD, FCG, PER, W64, NT>(a.box, (gp<const TV>)a.wL, (gp<TV>)a.r,
                                          (gp<TV>)a.z, (gp<const TD>)a.dinv,
                                          (TV)st->alpha, (int64_t)q * VCH, a.nG, q,
                                          nitems, part, sm);
}

// rz, rr per solve -> convergence / beta
__global__ void __launch_bounds__(RT)
    k_bbeta(CgState *st, const double *__restrict__ part,
            const int32_t *__restrict__ vbeg, int nitems) {
  __shared__ double sm[RT / 64];
  const int s = blockIdx.x;
  if (st[s].done != 0) return;
  double acc[2];
  strided_sums<2>(part, nitems, vbeg[s], vbeg[s + 1], acc);
  const double a = acc[0], b = acc[1];
  const double rz = block_sum<RT>(a, sm);
  const double rr = block_sum<RT>(b, sm);
  if (threadIdx.x == 0) {
    CgState &c = st[s];
    c.xupd = 1;  // this step's alpha is finite: x += alpha p follows
    c.it += 1;
    c.rr = rr;
    if (!isfinite(rr) || !isfinite(rz))
      c.done = 2;
    else if (rr <= c.tol2 * c.bb)
      c.done = 1;
    else if (c.it >= c.maxit)
      c.done = 3;
    else {
      c.beta = rz / c.rz;
      c.rz = rz;
    }
  }
}

// x += alpha p with this step's alpha (when k_bbeta found it finite, also
// on the step that converged), then p = z + beta p while the solve runs
template <class TV, bool NT>
__device__ __forceinline__ void p_chunk(gp<const TV> z, gp<TV> p, gp<TV> x, TV alpha,
                                        TV beta, bool run, int64_t start, int64_t nG) {
  const int64_t end = min(start + (int64_t)VCH, nG);
  constexpr int K = VCH / RT;
  const int64_t g0 = start + threadIdx.x;
  if (run && g0 + (K - 1) * RT < end) {
    // a whole chunk: every load of the thread's K nodes before any store
    // (the compiler cannot know that x, p and z do not overlap): 78 -> 67
    // us at 11.4M unique nodes in FP64.  NT: x and z stream non-temporally
    // (x is next read an iteration later, z not again); p (gathered by the
    // next operator) keeps the normal hint, so that it can stay in the
    // last-level cache
    TV pv[K], xv[K], zv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      pv[k] = p[g0 + k * RT];
      xv[k] = ld_h<NT>(x + g0 + k * RT);
      zv[k] = ld_h<NT>(z + g0 + k * RT);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      st_h<NT>(xv[k] + alpha * pv[k], x + g0 + k * RT);
      p[g0 + k * RT] = zv[k] + beta * pv[k];
    }
  } else if (run) {
    for (int64_t g = g0; g < end; g += RT) {
      const TV pv = p[g];
      x[g] = x[g] + alpha * pv;
      p[g] = z[g] + beta * pv;
    }
  } else {
    for (int64_t g = g0; g < end; g += RT) x[g] = x[g] + alpha * p[g];
  }
}

template <class TV, bool NT>
__global__ void __launch_bounds__(RT)
    k_bupdate_p(const BatchSolve *__restrict__ sds, const CgState *__restrict__ st,
                const VecItem *__restrict__ items, int nitems) {
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    const CgState &c = st[it.solve];
    if (c.xupd == 0) continue;  // uniform per item
    const BatchSolve &sd = sds[it.solve];
    p_chunk<TV, NT>(vec<TV>(sd, VZ), vec<TV>(sd, VP), vec<TV>(sd, VX), (TV)c.alpha,
                    (TV)c.beta, c.done == 0, it.start, sd.nG);
  }
}

// the same for the chunks of a single solve
template <class TV, class TD, bool NT>
__global__ void __launch_bounds__(RT)
    k_p_1(Vecs1<TV, TD> a, const CgState *__restrict__ st) {
  const CgState &c = *st;
  if (c.xupd == 0) return;
  p_chunk<TV, NT>((gp<const TV>)a.z, (gp<TV>)a.p, (gp<TV>)a.x, (TV)c.alpha, (TV)c.beta,
                  c.done == 0, (int64_t)blockIdx.x * VCH, a.nG);
}

// r = b - w (x0_zero: r = b and x = 0), z = dinv r, p = z; partials of
// (r, z), (r, r), (b, b)
template <class TV, class TD>
__global__ void __launch_bounds__(RT)
    k_binit(const BatchSolve *__restrict__ sds, const int32_t *__restrict__ active,
            const VecItem *__restrict__ items, int nitems,
            double *__restrict__ part, int x0_zero, int jac) {
  __shared__ double sm[RT / 64];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (!active[it.solve]) continue;
    const BatchSolve &sd = sds[it.solve];
    gp<const TV> b = vec<TV>(sd, VB), w = vec<TV>(sd, VW);
    gp<TV> x = vec<TV>(sd, VX), r = vec<TV>(sd, VR), z = vec<TV>(sd, VZ),
           p = vec<TV>(sd, VP);
    gp<const TD> dinv = dinv_of<TD>(sd, jac);
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT) {
      const TV bv = b[g];
      TV rv = bv;
      if (x0_zero)
        x[g] = TV(0);
      else
        rv = bv - w[g];
      const TV zv = (TV)(dinv[g] * rv);
      r[g] = rv;
      z[g] = zv;
      p[g] = zv;
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
      bb += (double)bv * (double)bv;
    }
    const double a = block_sum<RT>(rz, sm);
    const double c = block_sum<RT>(rr, sm);
    const double d = block_sum<RT>(bb, sm);
    if (threadIdx.x == 0) {
      part[q] = a;
      part[nitems + q] = c;
      part[2 * nitems + q] = d;
    }
  }
}

__global__ void __launch_bounds__(RT)
    k_binit_reduce(CgState *st, const double *__restrict__ part,
                   const int32_t *__restrict__ vbeg, int nitems,
                   const int32_t *__restrict__ active,
                   const int32_t *__restrict__ maxit, double tol2) {
  __shared__ double sm[RT / 64];
  const int s = blockIdx.x;
  CgState &c = st[s];
  if (!active[s]) {
    if (threadIdx.x == 0) {
      c.done = 4;
      c.it = 0;
      c.xupd = 0;
    }
    return;
  }
  double acc[3];
  strided_sums<3>(part, nitems, vbeg[s], vbeg[s + 1], acc);
  const double a = acc[0], b = acc[1], d = acc[2];
  const double rz = block_sum<RT>(a, sm);
  const double rr = block_sum<RT>(b, sm);
  const double bb = block_sum<RT>(d, sm);
  if (threadIdx.x == 0) {
    c.rz = rz;
    c.rr = rr;
    c.bb = bb;
    c.tol2 = tol2;
    c.it = 0;
    c.maxit = maxit[s];
    c.xupd = 0;
    c.alpha = c.beta = c.pw = 0.0;
    if (!isfinite(rr) || !isfinite(rz))
      c.done = 2;
    else if (rr <= tol2 * bb)
      c.done = 1;
    else if (c.maxit <= 0)
      c.done = 3;
    else
      c.done = 0;
  }
}

// FP64 residual r = b - w (stored), partials (r, r), (b, b)
__global__ void __launch_bounds__(RT)
    k_bresidual(const BatchSolve *__restrict__ sds,
                const int32_t *__restrict__ active,
                const VecItem *__restrict__ items, int nitems,
                double *__restrict__ part) {
  __shared__ double sm[RT / 64];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (!active[it.solve]) continue;
    const BatchSolve &sd = sds[it.solve];
    gp<const double> b = vec<double>(sd, VB), w = vec<double>(sd, VW);
    gp<double> r = vec<double>(sd, VR);
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    double rr = 0.0, bb = 0.0;
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT) {
      const double rv = b[g] - w[g];
      r[g] = rv;
      rr += rv * rv;
      bb += b[g] * b[g];
    }
    const double a = block_sum<RT>(rr, sm);
    const double c = block_sum<RT>(bb, sm);
    if (threadIdx.x == 0) {
      part[q] = a;
      part[nitems + q] = c;
    }
  }
}

// out[2 s], out[2 s + 1] = sums of the two partial rows over solve s
__global__ void __launch_bounds__(RT)
    k_breduce2(const double *__restrict__ part, const int32_t *__restrict__ vbeg,
               int nitems, const int32_t *__restrict__ active, double *out) {
  __shared__ double sm[RT / 64];
  const int s = blockIdx.x;
  if (!active[s]) return;
  double acc[2];
  strided_sums<2>(part, nitems, vbeg[s], vbeg[s + 1], acc);
  const double a = acc[0], b = acc[1];
  const double s0 = block_sum<RT>(a, sm);
  const double s1 = block_sum<RT>(b, sm);
  if (threadIdx.x == 0) {
    out[2 * s] = s0;
    out[2 * s + 1] = s1;
  }
}

// inner right-hand side b32 = r64 * scale_s; x64 += d32 / scale_s
__global__ void __launch_bounds__(RT)
    k_bscale_cast(const BatchSolve *__restrict__ sds,
                  const int32_t *__restrict__ active,
                  const double *__restrict__ scale,
                  const VecItem *__restrict__ items, int nitems) {
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (!active[it.solve]) continue;
    const BatchSolve &sd = sds[it.solve];
    gp<const double> r = vec<double>(sd, VR);
    gp<float> b = vec<float>(sd, VB);
    const double sc = scale[it.solve];
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT)
      b[g] = (float)(r[g] * sc);
  }
}

__global__ void __launch_bounds__(RT)
    k_baxpy_mixed(const BatchSolve *__restrict__ sds,
                  const int32_t *__restrict__ active,
                  const double *__restrict__ scale,
                  const VecItem *__restrict__ items, int nitems) {
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (!active[it.solve]) continue;
    const BatchSolve &sd = sds[it.solve];
    gp<double> x = vec<double>(sd, VX);
    gp<const float> d = vec<float>(sd, VX);
    const double inv = 1.0 / scale[it.solve];
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT)
      x[g] += inv * (double)d[g];
  }
}

// z = dinv r + c with c the coarse correction on unique nodes (cG); partials
// (r, z), (z, w), (r, r).  skip_done = 0 during initialisation.
template <class TV, class TD>
__global__ void __launch_bounds__(RT)
    k_bprec_learned(const BatchSolve *__restrict__ sds,
                    const CgState *__restrict__ st,
                    const VecItem *__restrict__ items, int nitems,
                    const float *__restrict__ cG, double *__restrict__ part,
                    int skip_done) {
  __shared__ double sm[RT / 64];
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (skip_done && st[it.solve].done != 0) continue;
    const BatchSolve &sd = sds[it.solve];
    gp<const TV> r = vec<TV>(sd, VR), w = vec<TV>(sd, VW);
    gp<TV> z = vec<TV>(sd, VZ);
    gp<const TD> dinv = dinv_of<TD>(sd, 1);
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    double rz = 0.0, zw = 0.0, rr = 0.0;
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT) {
      const TV rv = r[g];
      // dinv is 0 on the Dirichlet boundary, where cG is 0 too
      const TV zv = (TV)(dinv[g] * rv) + (TV)cG[g];
      z[g] = zv;
      rz += (double)rv * (double)zv;
      zw += (double)zv * (double)w[g];
      rr += (double)rv * (double)rv;
    }
    const double a1 = block_sum<RT>(rz, sm);
    const double a2 = block_sum<RT>(zw, sm);
    const double a3 = block_sum<RT>(rr, sm);
    if (threadIdx.x == 0) {
      part[q] = a1;
      part[nitems + q] = a2;
      part[2 * nitems + q] = a3;
    }
  }
}

// flexible CG (Notay's, one stored direction): beta = -(z, A p) / (p, A p),
// convergence on (r, r), for one solve whose correction step stored its
// element terms of (r, c) and (c, w) in epart ([2][E]): (r, z) and (z, w)
// are the partials of the r update plus those terms
__global__ void __launch_bounds__(RT)
    k_bbeta_fcg_e(CgState *st, const double *__restrict__ part, int nitems,
                  const double *__restrict__ epart, int E) {
  __shared__ double sm[RT / 64];
  CgState &cs = st[0];
  if (cs.done != 0) return;
  double acc[3], ea[2];
  strided_sums<3>(part, nitems, 0, nitems, acc);
  strided_sums<2>(epart, E, 0, E, ea);
  const double rz = block_sum<RT>(acc[0] + ea[0], sm);
  const double zw = block_sum<RT>(acc[1] + ea[1], sm);
  const double rr = block_sum<RT>(acc[2], sm);
  if (threadIdx.x == 0) {
    cs.xupd = 1;  // this step's alpha is finite: x += alpha p follows
    cs.it += 1;
    cs.rr = rr;
    if (!isfinite(rr) || !isfinite(rz) || !isfinite(zw))
      cs.done = 2;
    else if (rr <= cs.tol2 * cs.bb)
      cs.done = 1;
    else if (cs.it >= cs.maxit)
      cs.done = 3;
    else {
      cs.beta = -zw / cs.pw;
      cs.rz = rz;
    }
  }
}

// start of flexible CG: rz from the partials, p = z
__global__ void __launch_bounds__(RT)
    k_bfcg_start(CgState *st, const double *__restrict__ part,
                 const int32_t *__restrict__ vbeg) {
  __shared__ double sm[RT / 64];
  const int s = blockIdx.x;
  double acc[1];
  strided_sums<1>(part, 0, vbeg[s], vbeg[s + 1], acc);
  const double rz = block_sum<RT>(acc[0], sm);
  if (threadIdx.x == 0) {
    st[s].rz = rz;
    if (st[s].done == 0 && !isfinite(rz)) st[s].done = 2;
  }
}

template <class TV>
__global__ void __launch_bounds__(RT)
    k_bcopy_zp(const BatchSolve *__restrict__ sds, const CgState *__restrict__ st,
               const VecItem *__restrict__ items, int nitems) {
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const VecItem it = items[q];
    if (st[it.solve].done != 0) continue;
    const BatchSolve &sd = sds[it.solve];
    gp<const TV> z = vec<TV>(sd, VZ);
    gp<TV> p = vec<TV>(sd, VP);
    const int64_t end = min(it.start + (int64_t)VCH, sd.nG);
    for (int64_t g = it.start + threadIdx.x; g < end; g += RT) p[g] = z[g];
  }
}

__global__ void k_first_copy(int64_t nG, const int32_t *__restrict__ off,
                             const int32_t *__restrict__ perm,
                             const double *__restrict__ vL,
                             double *__restrict__ vG) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nG) vG[g] = vL[perm[off[g]]];
}

__global__ void k_scatter(int64_t nL, const int32_t *__restrict__ l2g,
                          const double *__restrict__ vG, double *__restrict__ vL) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nL) vL[l] = vG[l2g[l]];
}

__global__ void k_unmask(int64_t nG, const uint8_t *__restrict__ gmask,
                         double *__restrict__ o64, float *__restrict__ o32) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nG) {
    o64[g] = gmask[g] ? 0.0 : 1.0;
    if (o32 != nullptr) o32[g] = gmask[g] ? 0.0f : 1.0f;
  }
}

// --------------------------------------------------------------------------
// per-handle solver vectors
// --------------------------------------------------------------------------
struct Workspace {
  DevBuf v64[NVEC], v32[NVEC], one64, one32;
  DevBuf edot;  // element energies of the last operator application
  bool ready = false;
  sem_batch *single = nullptr;  // the handle as a batch of one
};

static unsigned nblk(int64_t n) { return (unsigned)((n + RT - 1) / RT); }

static void ensure_vectors(sem_handle *h) {
  if (h->ws == nullptr) h->ws = new Workspace();
  Workspace *W = h->ws;
  if (W->ready) return;
  for (int v = 0; v < NVEC; ++v) {
    const int64_t n = v == VWL ? h->nL : h->nG;
    W->v64[v].alloc(n * sizeof(double));
    W->v32[v].alloc(n * sizeof(float));
  }
  W->one64.alloc(h->nG * sizeof(double));
  W->one32.alloc(h->nG * sizeof(float));
  W->edot.alloc(h->E * sizeof(double));
  hipLaunchKernelGGL(k_unmask, dim3(nblk(h->nG)), dim3(RT), 0, 0, h->nG,
                     h->gmask.as<uint8_t>(), W->one64.as<double>(),
                     W->one32.as<float>());
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipDeviceSynchronize());
  W->ready = true;
}

}  // namespace sem

// --------------------------------------------------------------------------
// batches
// --------------------------------------------------------------------------
struct sem_batch {
  std::vector<sem_handle *> hs;
  int n = 0;
  int nset = 0;                 // order set the operator kernel is built for
  std::vector<int> orders;      // n1 per solve
  std::vector<sem::BatchSolve> hsd;  // host copies of the solve descriptors
  bool periodic = false;        // a solve of the batch has a periodic direction
  bool wide = false;            // a solve's local indices need 64 bits
  int64_t sum_nG = 0, sum_nL = 0;  // unique and local nodes of all solves
  sem::DevBuf sds, st, vitems, vbeg, part, red, active, maxit, scale;
  sem::DevBuf axitems[3];       // per block size 64 / 128 / 256
  int n_ax[3] = {0, 0, 0};
  int n_vi = 0;
  // The lists of the CG iteration kernels, compacted to the running solves
  // as solves finish (run_cg rebuilds them whenever the running solves hold
  // at most half of the listed vector chunks): each running solve keeps its
  // items in their order, so its partial sums are added as before and its
  // bits do not change.  Built from host copies of the full lists.
  sem::DevBuf vitems_c, vbeg_c, axitems_c[3];
  int n_vi_c = 0, n_ax_c[3] = {0, 0, 0};
  bool compact = false;         // the iteration kernels use the compacted lists
  int list_ver = 0;             // version of the compacted lists
  std::vector<sem::VecItem> h_vis;
  std::vector<sem::AxItem> h_ax[3];
  std::vector<int32_t> h_vbeg, h_axbeg[3];  // per-solve item ranges
  int bs[5] = {128, 64, 64, 256, 256};  // operator block size per precision
  int gmul[5] = {0, 0, 0, 0, 0};  // persistent grid = 256 CUs x gmul (0: 1 item/WG)
  sem::CgState *host_st = nullptr;
  double *host_red = nullptr;
  int32_t *host_i = nullptr;    // staging for active / maxit
  double *host_d = nullptr;     // staging for scale
  // false for a batch laid out in caller-provided memory: host_* then point
  // to the inline arrays below and s is the caller's stream (none owned)
  bool owned = true;
  sem::CgState inl_st[1];
  double inl_red[2], inl_d[1];
  int32_t inl_i[1];
  hipStream_t s = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, fence = nullptr;
  struct GraphEntry {
    int prec, k, jac, mode, ver;  // ver: list version (0: the full lists)
    hipGraphExec_t exec;
  };
  // snapshot recording of solve 0 (training data), FP64 unique vectors
  double *snap_x = nullptr, *snap_r = nullptr;
  int snap_max = 0, snap_count = 0;
  std::vector<GraphEntry> graphs;
  bool tuned = false;
  ~sem_batch() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (owned) {
      if (host_st) (void)hipHostFree(host_st);
      if (host_red) (void)hipHostFree(host_red);
      if (host_i) (void)hipHostFree(host_i);
      if (host_d) (void)hipHostFree(host_d);
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (fence) (void)hipEventDestroy(fence);
    if (owned && s) (void)hipStreamDestroy(s);
  }
};

namespace sem {

static int bs_slot(int bs) { return bs == 64 ? 0 : bs == 128 ? 1 : 2; }

// the device descriptor of solve q: the handle's operator arrays and the
// given solver vectors
static BatchSolve describe(sem_handle *h, int q, void *const v64[NVEC],
                           void *const v32[NVEC], const double *one64,
                           const float *one32, double *edot) {
  BatchSolve d;
  memset(&d, 0, sizeof d);
  d.N1 = h->n1;
  d.solve = q;
  d.E = h->E;
  d.nL = h->nL;
  d.nG = h->nG;
  d.box = make_box(h->N, h->ex, h->ey, h->ez, h->dirichlet, h->periodic);
  d.G64 = h->G64.p;
  d.G32 = h->G32.p;
  d.G16 = h->G16.p;
  d.D64 = h->D64.p;
  d.D32 = h->D32.p;
  d.D16hi = h->D16hi.p;
  d.D16lo = h->D16lo.p;
  d.H16 = h->has_mass ? h->H16.p : nullptr;
  d.dinv64 = h->dinv_G.as<double>();
  d.dinv32 = h->dinv_G32.as<float>();
  d.one64 = one64;
  d.one32 = one32;
  for (int v = 0; v < NVEC; ++v) {
    d.v64[v] = v64[v];
    d.v32[v] = v32[v];
  }
  d.edot = edot;
  return d;
}

sem_batch *batch_create(sem_handle *const *hs, int n) {
  if (n < 1) fail(SEM_ERR_ARG, "batch: need at least one handle");
  std::set<int> orders;
  for (int q = 0; q < n; ++q) {
    if (hs[q] == nullptr) fail(SEM_ERR_ARG, "batch: null handle");
    if (hs[q]->nL >= (int64_t)INT32_MAX) fail(SEM_ERR_ARG, "batch: solve too large");
    orders.insert(hs[q]->n1);
    for (int r = 0; r < q; ++r)
      if (hs[r] == hs[q]) fail(SEM_ERR_ARG, "batch: a handle appears twice");
    // the persistent batched operator has no mass term; a single solve runs
    // the gathered single-solve operator, which has
    if (n > 1 && hs[q]->has_mass)
      fail(SEM_ERR_ARG, "batch: solves with a mass term (alpha != 0) must be "
                        "solved one at a time");
  }
  int nset;
  if (orders.size() == 1)
    nset = *orders.begin();
  else {
    for (int o : orders)
      if (o != 4 && o != 6 && o != 8)
        fail(SEM_ERR_ARG, "batch: mixed orders must be within N in {3, 5, 7}");
    nset = AX_SET_468;
  }
  sem_batch *b = new sem_batch();
  try {
    b->hs.assign(hs, hs + n);
    b->n = n;
    b->nset = nset;
    // default operator block sizes hold every column of an element
    for (int &x : b->bs) x = std::max(x, bax_min_block(nset));
    std::vector<BatchSolve> sds(n);
    std::vector<VecItem> vis;
    std::vector<int32_t> vbeg(n + 1);
    for (int q = 0; q < n; ++q) {
      sem_handle *h = hs[q];
      ensure_vectors(h);
      Workspace *W = h->ws;
      void *v64[NVEC], *v32[NVEC];
      for (int v = 0; v < NVEC; ++v) {
        v64[v] = W->v64[v].p;
        v32[v] = W->v32[v].p;
      }
      sds[q] = describe(h, q, v64, v32, W->one64.as<double>(),
                        W->one32.as<float>(), W->edot.as<double>());
      if (h->periodic != 0) b->periodic = true;
      if (h->nL > (int64_t)UINT32_MAX) b->wide = true;
      b->sum_nG += h->nG;
      b->sum_nL += h->nL;
      vbeg[q] = (int32_t)vis.size();
      for (int64_t g = 0; g < h->nG; g += VCH) vis.push_back({q, 0, g});
      b->orders.push_back(h->n1);
    }
    vbeg[n] = (int32_t)vis.size();
    b->n_vi = (int)vis.size();
    const int bss[3] = {64, 128, 256};
    for (int k = 0; k < 3; ++k) {
      std::vector<AxItem> ax;
      b->h_axbeg[k].assign(n + 1, 0);
      for (int q = 0; q < n; ++q) {
        b->h_axbeg[k][q] = (int32_t)ax.size();
        const int epb = bax_elements_per_tile(bss[k], hs[q]->n1);
        for (int64_t e = 0; e < hs[q]->E; e += epb) ax.push_back({q, 0, e});
      }
      b->h_axbeg[k][n] = (int32_t)ax.size();
      b->n_ax[k] = (int)ax.size();
      b->axitems[k].alloc(ax.size() * sizeof(AxItem));
      SEM_HIP(hipMemcpy(b->axitems[k].p, ax.data(), ax.size() * sizeof(AxItem),
                        hipMemcpyHostToDevice));
      if (n > 1) b->axitems_c[k].alloc(ax.size() * sizeof(AxItem));
      b->h_ax[k] = std::move(ax);
    }
    if (n > 1) {
      b->vitems_c.alloc(vis.size() * sizeof(VecItem));
      b->vbeg_c.alloc((n + 1) * sizeof(int32_t));
    }
    b->h_vis = vis;
    b->h_vbeg = vbeg;
    b->hsd = sds;
    b->sds.alloc(n * sizeof(BatchSolve));
    SEM_HIP(hipMemcpy(b->sds.p, sds.data(), n * sizeof(BatchSolve),
                      hipMemcpyHostToDevice));
    b->vitems.alloc(vis.size() * sizeof(VecItem));
    SEM_HIP(hipMemcpy(b->vitems.p, vis.data(), vis.size() * sizeof(VecItem),
                      hipMemcpyHostToDevice));
    b->vbeg.alloc((n + 1) * sizeof(int32_t));
    SEM_HIP(hipMemcpy(b->vbeg.p, vbeg.data(), (n + 1) * sizeof(int32_t),
                      hipMemcpyHostToDevice));
    b->part.alloc(3 * (size_t)b->n_vi * sizeof(double));
    b->st.alloc(n * sizeof(CgState));
    b->red.alloc(2 * n * sizeof(double));
    b->active.alloc(n * sizeof(int32_t));
    b->maxit.alloc(n * sizeof(int32_t));
    b->scale.alloc(n * sizeof(double));
    SEM_HIP(hipHostMalloc((void **)&b->host_st, n * sizeof(CgState), 0));
    SEM_HIP(hipHostMalloc((void **)&b->host_red, 2 * n * sizeof(double), 0));
    SEM_HIP(hipHostMalloc((void **)&b->host_i, n * sizeof(int32_t), 0));
    SEM_HIP(hipHostMalloc((void **)&b->host_d, n * sizeof(double), 0));
    SEM_HIP(hipEventCreate(&b->ev0));
    SEM_HIP(hipEventCreate(&b->ev1));
    SEM_HIP(hipEventCreateWithFlags(&b->fence, hipEventDisableTiming));
    SEM_HIP(hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking));
    SEM_HIP(hipDeviceSynchronize());
  } catch (...) {
    delete b;
    throw;
  }
  return b;
}

void batch_destroy(sem_batch *b) { delete b; }

void destroy_ws(sem_handle *h) {
  if (h->ws == nullptr) return;
  delete h->ws->single;
  delete h->ws;
  h->ws = nullptr;
}

// --------------------------------------------------------------------------
// launches of one batch
// --------------------------------------------------------------------------
// one workgroup per chunk of unique nodes: with fewer, persistent
// workgroups the last round of chunks runs on part of the chip (FP64
// assembly + r update at 11.4M unique nodes: 114 -> 104 us)
static int vec_grid(const sem_batch *b) { return b->n_vi; }

// Streaming (non-temporal) hints on the solver's vectors and operator output
// when the batch's vectors (about five unique-node vectors and the E-vector,
// of `tv` bytes per value) exceed half of the 256 MB last-level cache: their
// next use is then an iteration away and they would not stay cached anyway;
// smaller solves keep the normal hints and their vectors stay cached.
constexpr double NT_BYTES = 128.0 * 1024 * 1024;
static int stream_vectors(const sem_batch *b, size_t tv) {
  return (double)tv * (5.0 * (double)b->sum_nG + (double)b->sum_nL) > NT_BYTES ? 1 : 0;
}

// the work lists of the CG iteration kernels: compacted while run_cg has
// built them, else the full lists
static const VecItem *it_vitems(const sem_batch *b) {
  return b->compact ? b->vitems_c.as<VecItem>() : b->vitems.as<VecItem>();
}
static int it_nvi(const sem_batch *b) { return b->compact ? b->n_vi_c : b->n_vi; }
static const int32_t *it_vbeg(const sem_batch *b) {
  return b->compact ? b->vbeg_c.as<int32_t>() : b->vbeg.as<int32_t>();
}
static const AxItem *it_axitems(const sem_batch *b, int k) {
  return b->compact ? b->axitems_c[k].as<AxItem>() : b->axitems[k].as<AxItem>();
}
static int it_nax(const sem_batch *b, int k) { return b->compact ? b->n_ax_c[k] : b->n_ax[k]; }

// launch an assembly kernel in its variant for the batch's boxes: with a
// periodic direction in any solve (PER_ = true) or without
#define SEM_PER_LAUNCH(B, KERNEL, ...)                     \
  do {                                                     \
    if ((B)->periodic) {                                   \
      constexpr bool PER_ = true;                          \
      hipLaunchKernelGGL(KERNEL, __VA_ARGS__);             \
    } else {                                               \
      constexpr bool PER_ = false;                         \
      hipLaunchKernelGGL(KERNEL, __VA_ARGS__);             \
    }                                                      \
  } while (0)

// launch a vector kernel in its variant with (NT_ = true) or without the
// streaming hints (stream_vectors)
#define SEM_NT_LAUNCH(NT, KERNEL, ...)                     \
  do {                                                     \
    if (NT) {                                              \
      constexpr bool NT_ = true;                           \
      hipLaunchKernelGGL(KERNEL, __VA_ARGS__);             \
    } else {                                               \
      constexpr bool NT_ = false;                          \
      hipLaunchKernelGGL(KERNEL, __VA_ARGS__);             \
    }                                                      \
  } while (0)

// the same, with W64_ = true when some local index of the batch needs more
// than 32 bits
#define SEM_ASM_LAUNCH(B, KERNEL, ...)                     \
  do {                                                     \
    if ((B)->wide) {                                       \
      constexpr bool W64_ = true;                          \
      SEM_PER_LAUNCH(B, KERNEL, __VA_ARGS__);              \
    } else {                                               \
      constexpr bool W64_ = false;                         \
      SEM_PER_LAUNCH(B, KERNEL, __VA_ARGS__);              \
    }                                                      \
  } while (0)

// the same, also choosing the variant with (NT_ = true) or without the
// streaming hints
#define SEM_ASM_NT_LAUNCH(B, NT, KERNEL, ...)              \
  do {                                                     \
    if (NT) {                                              \
      constexpr bool NT_ = true;                           \
      SEM_ASM_LAUNCH(B, KERNEL, __VA_ARGS__);              \
    } else {                                               \
      constexpr bool NT_ = false;                          \
      SEM_ASM_LAUNCH(B, KERNEL, __VA_ARGS__);              \
    }                                                      \
  } while (0)

// the operator of every solve of the batch, w_L = A_L Q v_src into VWL;
// edot: the single-solve kernel also stores the element energies (the
// batched kernel always does)
static void bax(sem_batch *b, int prec, int src, int dst, int skip_done,
                bool edot = false) {
  if (prec == SEM_BF16_MFMA || prec == SEM_BF16_PLAIN_D) {
    // matrix-core operator: tiles of the 256-thread item list, one order
    if (b->nset < 2 || b->nset > 9)
      fail(SEM_ERR_ARG, "solve: the matrix-core operator needs solves of one "
                        "order N <= 8");
    if (b->n == 1) {  // a single solve: every argument passed in
      const BatchSolve &d = b->hsd[0];
      const int32_t *stop =
          skip_done ? &b->st.as<CgState>()[0].done : (const int32_t *)nullptr;
      launch_ax_mfma_solve(d.N1 - 1, prec == SEM_BF16_MFMA, d.E, (const uint16_t *)d.D16hi,
                           (const uint16_t *)d.D16lo, (const uint16_t *)d.G16,
                           (const uint16_t *)d.H16, (const float *)d.v32[src],
                           (float *)d.v32[dst], d.box, stop, edot ? d.edot : nullptr, b->s);
      return;
    }
    const int k = bs_slot(256);
    launch_bax_mfma(b->nset, prec == SEM_BF16_MFMA, b->sds.as<BatchSolve>(),
                    b->st.as<CgState>(), it_axitems(b, k), it_nax(b, k),
                    bax_elements_per_tile(256, b->nset), it_nax(b, k), src, dst,
                    skip_done, edot, b->s);
    return;
  }
  if (b->n == 1) {
    // a single solve: the operator with every argument in registers
    sem_handle *h = b->hs[0];
    const BatchSolve &d = b->hsd[0];
    const bool f64 = prec == SEM_FP64;
    const void *G = f64 ? h->G64.p : prec == SEM_FP32 ? h->G32.p : h->G16.p;
    const void *H = !h->has_mass ? nullptr
                    : f64        ? h->H64.p
                    : prec == SEM_FP32 ? h->H32.p
                                       : h->H16.p;
    const void *D = f64 ? h->D64.p : h->D32.p;
    const void *u = f64 ? d.v64[src] : d.v32[src];
    void *w = f64 ? d.v64[dst] : d.v32[dst];
    const int32_t *stop =
        skip_done ? &b->st.as<CgState>()[0].done : (const int32_t *)nullptr;
    launch_ax_solve(h->N, prec, h->E, D, G, H, u, w,
                    make_box(h->N, h->ex, h->ey, h->ez, h->dirichlet, h->periodic), stop,
                    edot ? d.edot : nullptr, stream_vectors(b, f64 ? 8 : 4) != 0, b->s);
    return;
  }
  const int bs = b->bs[prec];
  const int k = bs_slot(bs);
  const int n = it_nax(b, k);
  const int grid = b->gmul[prec] > 0 ? std::min(n, 256 * b->gmul[prec]) : n;
  launch_bax(prec, bs, b->nset, b->sds.as<BatchSolve>(), b->st.as<CgState>(),
             it_axitems(b, k), n, grid, src, dst, skip_done, b->s);
}

// the single-solve kernels' view of the batch's one solve
template <class TV, class TD>
static Vecs1<TV, TD> vecs1(const sem_batch *b, int jac) {
  const BatchSolve &d = b->hsd[0];
  auto v = [&](int i) { return (TV *)(sizeof(TV) == 8 ? d.v64[i] : d.v32[i]); };
  Vecs1<TV, TD> a;
  a.box = d.box;
  a.nG = d.nG;
  a.wL = v(VWL);
  a.r = v(VR);
  a.z = v(VZ);
  a.p = v(VP);
  a.x = v(VX);
  a.dinv = (const TD *)(sizeof(TD) == 8 ? (jac ? (const void *)d.dinv64 : d.one64)
                                        : (jac ? (const void *)d.dinv32 : d.one32));
  return a;
}

template <class TV, class TD>
static void iteration_t(sem_batch *b, int prec, int jac) {
  const BatchSolve *sds = b->sds.as<BatchSolve>();
  CgState *st = b->st.as<CgState>();
  const VecItem *vi = it_vitems(b);
  double *part = b->part.as<double>();
  const int32_t *vbeg = it_vbeg(b);
  const int nv = it_nvi(b), g = nv, n = b->n;
  // (p, A p) from the operator's element energies (every operator form, the
  // matrix-core one included, stores them)
  const bool nt = stream_vectors(b, sizeof(TV)) != 0;
  bax(b, prec, VP, VWL, 1, true);
  hipLaunchKernelGGL(k_balpha_e, dim3(n), dim3(AT), 0, b->s, sds, st);
  if (b->n == 1)
    SEM_ASM_NT_LAUNCH(b, nt, (k_xr_asm_1<TV, TD, false, PER_, W64_, NT_>), dim3(nv),
                      dim3(RT), 0, b->s, vecs1<TV, TD>(b, jac), st, nv, part);
  else
    SEM_ASM_NT_LAUNCH(b, nt, (k_bupdate_xr_asm<TV, TD, false, PER_, W64_, NT_>), dim3(g),
                      dim3(RT), 0, b->s, sds, st, vi, nv, part, jac);
  hipLaunchKernelGGL(k_bbeta, dim3(n), dim3(RT), 0, b->s, st, part, vbeg, nv);
  if (b->n == 1)
    SEM_NT_LAUNCH(nt, (k_p_1<TV, TD, NT_>), dim3(nv), dim3(RT), 0, b->s,
                  vecs1<TV, TD>(b, jac), st);
  else
    SEM_NT_LAUNCH(nt, (k_bupdate_p<TV, NT_>), dim3(g), dim3(RT), 0, b->s, sds, st, vi, nv);
  SEM_HIP(hipGetLastError());
}

// flexible CG with the learned correction (single solves): (p, A p) from the
// operator's element energies; the r update forms the assembled w, z = dinv r
// and the partials of (r, z), (z, w), (r, r); the correction step adds c to
// z on the element interiors and stores the element terms of (r, c) and
// (c, w)
template <class TV, class TD>
static void iteration_fcg_t(sem_batch *b, int prec) {
  CgState *st = b->st.as<CgState>();
  double *part = b->part.as<double>();
  const int nv = b->n_vi, n = b->n;
  sem_handle *h = b->hs[0];
  const bool f32 = sizeof(TV) == 4;
  const bool nt = stream_vectors(b, sizeof(TV)) != 0;
  bax(b, prec, VP, VWL, 1, true);
  hipLaunchKernelGGL(k_balpha_e, dim3(n), dim3(AT), 0, b->s, b->sds.as<BatchSolve>(), st);
  SEM_ASM_NT_LAUNCH(b, nt, (k_xr_asm_1<TV, TD, true, PER_, W64_, NT_>), dim3(nv), dim3(RT),
                    0, b->s, vecs1<TV, TD>(b, 1), st, nv, part);
  const BatchSolve &d = b->hsd[0];
  learn_apply_fused(h, f32 ? d.v32[VR] : d.v64[VR], f32 ? d.v32[VZ] : d.v64[VZ],
                    f32 ? d.v32[VWL] : d.v64[VWL], f32, b->s);
  hipLaunchKernelGGL(k_bbeta_fcg_e, dim3(1), dim3(RT), 0, b->s, st, part, nv,
                     learn_epart(h), (int)h->E);
  SEM_NT_LAUNCH(nt, (k_p_1<TV, TD, NT_>), dim3(nv), dim3(RT), 0, b->s, vecs1<TV, TD>(b, 1),
                st);
  SEM_HIP(hipGetLastError());
}

// mode 0: PCG with the `jac` preconditioner; mode 1: flexible CG with the
// learned correction
static void iteration(sem_batch *b, int prec, int jac, int mode = 0) {
  if (mode == 1) {
    if (prec == SEM_FP64)
      iteration_fcg_t<double, double>(b, prec);
    else
      iteration_fcg_t<float, float>(b, prec);
    return;
  }
  if (prec == SEM_FP64)
    iteration_t<double, double>(b, prec, jac);
  else
    iteration_t<float, float>(b, prec, jac);
}

float *learn_cg(sem_handle *h);

// after init(): replace z by the learned preconditioner, p = z, rz
static void init_fcg(sem_batch *b, int prec) {
  const BatchSolve *sds = b->sds.as<BatchSolve>();
  CgState *st = b->st.as<CgState>();
  const VecItem *vi = b->vitems.as<VecItem>();
  double *part = b->part.as<double>();
  const int g = vec_grid(b), nv = b->n_vi;
  sem_handle *h = b->hs[0];
  const bool f32 = prec != SEM_FP64;
  learn_apply(h, f32 ? b->hsd[0].v32[VR] : b->hsd[0].v64[VR], f32, b->s);
  if (f32) {
    hipLaunchKernelGGL((k_bprec_learned<float, float>), dim3(g), dim3(RT), 0, b->s,
                       sds, st, vi, nv, learn_cg(h), part, 0);
  } else {
    hipLaunchKernelGGL((k_bprec_learned<double, double>), dim3(g), dim3(RT), 0,
                       b->s, sds, st, vi, nv, learn_cg(h), part, 0);
  }
  hipLaunchKernelGGL(k_bfcg_start, dim3(b->n), dim3(RT), 0, b->s, st, part,
                     b->vbeg.as<int32_t>());
  if (f32)
    hipLaunchKernelGGL((k_bcopy_zp<float>), dim3(g), dim3(RT), 0, b->s, sds, st, vi,
                       nv);
  else
    hipLaunchKernelGGL((k_bcopy_zp<double>), dim3(g), dim3(RT), 0, b->s, sds, st,
                       vi, nv);
  SEM_HIP(hipGetLastError());
}

// initial residual and state for the active solves; the vector set of `prec`
static void init(sem_batch *b, int prec, int jac, bool x0_zero, double tol2) {
  const BatchSolve *sds = b->sds.as<BatchSolve>();
  const VecItem *vi = b->vitems.as<VecItem>();
  double *part = b->part.as<double>();
  const int g = vec_grid(b), nv = b->n_vi;
  const int32_t *act = b->active.as<int32_t>();
  if (!x0_zero) {
    // w = A x (FP64 only)
    bax(b, SEM_FP64, VX, VWL, 0);
    SEM_PER_LAUNCH(b, (k_bassemble<double, false, PER_>), dim3(g), dim3(RT), 0, b->s,
                       sds, b->st.as<CgState>(), vi, nv, part, 0);
  }
  if (prec == SEM_FP64)
    hipLaunchKernelGGL((k_binit<double, double>), dim3(g), dim3(RT), 0, b->s, sds,
                       act, vi, nv, part, x0_zero ? 1 : 0, jac);
  else
    hipLaunchKernelGGL((k_binit<float, float>), dim3(g), dim3(RT), 0, b->s, sds,
                       act, vi, nv, part, x0_zero ? 1 : 0, jac);
  hipLaunchKernelGGL(k_binit_reduce, dim3(b->n), dim3(RT), 0, b->s,
                     b->st.as<CgState>(), part, b->vbeg.as<int32_t>(), nv, act,
                     b->maxit.as<int32_t>(), tol2);
  SEM_HIP(hipGetLastError());
}

// FP64 true residuals of the active solves: host_red[2s] = ||b - A x||^2,
// host_red[2s+1] = ||b||^2; r stored in VR
static void residual(sem_batch *b) {
  const BatchSolve *sds = b->sds.as<BatchSolve>();
  const VecItem *vi = b->vitems.as<VecItem>();
  double *part = b->part.as<double>();
  const int g = vec_grid(b), nv = b->n_vi;
  const int32_t *act = b->active.as<int32_t>();
  bax(b, SEM_FP64, VX, VWL, 0);
  SEM_PER_LAUNCH(b, (k_bassemble<double, false, PER_>), dim3(g), dim3(RT), 0, b->s, sds,
                     b->st.as<CgState>(), vi, nv, part, 0);
  hipLaunchKernelGGL(k_bresidual, dim3(g), dim3(RT), 0, b->s, sds, act, vi, nv,
                     part);
  hipLaunchKernelGGL(k_breduce2, dim3(b->n), dim3(RT), 0, b->s, part,
                     b->vbeg.as<int32_t>(), nv, act, b->red.as<double>());
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipMemcpyAsync(b->host_red, b->red.p, 2 * b->n * sizeof(double),
                         hipMemcpyDeviceToHost, b->s));
  SEM_HIP(hipStreamSynchronize(b->s));
}

static void upload_active(sem_batch *b, const std::vector<int> &act,
                          const std::vector<int> &maxit) {
  for (int q = 0; q < b->n; ++q) b->host_i[q] = act[q];
  SEM_HIP(hipMemcpyAsync(b->active.p, b->host_i, b->n * sizeof(int32_t),
                         hipMemcpyHostToDevice, b->s));
  SEM_HIP(hipStreamSynchronize(b->s));
  for (int q = 0; q < b->n; ++q) b->host_i[q] = maxit[q];
  SEM_HIP(hipMemcpyAsync(b->maxit.p, b->host_i, b->n * sizeof(int32_t),
                         hipMemcpyHostToDevice, b->s));
  SEM_HIP(hipStreamSynchronize(b->s));
}

static hipGraphExec_t get_graph(sem_batch *b, int prec, int K, int jac,
                                int mode) {
  const int ver = b->compact ? b->list_ver : 0;
  for (auto &g : b->graphs)
    if (g.prec == prec && g.k == K && g.jac == jac && g.mode == mode && g.ver == ver)
      return g.exec;
  hipGraph_t graph;
  SEM_HIP(hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal));
  try {
    for (int q = 0; q < K; ++q) iteration(b, prec, jac, mode);
  } catch (...) {
    hipGraph_t dummy;
    (void)hipStreamEndCapture(b->s, &dummy);
    throw;
  }
  SEM_HIP(hipStreamEndCapture(b->s, &graph));
  hipGraphExec_t exec;
  SEM_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  SEM_HIP(hipGraphDestroy(graph));
  b->graphs.push_back({prec, K, jac, mode, ver, exec});
  return exec;
}

// rebuild the iteration kernels' lists from the solves still running
// (host_st as last polled), when they hold at most half of the vector
// chunks of the lists in use; earlier compacted graphs are dropped
static void maybe_compact(sem_batch *b) {
  if (b->n < 2 || b->h_vis.empty()) return;
  int64_t run_items = 0;
  for (int q = 0; q < b->n; ++q)
    if (b->host_st[q].done == 0) run_items += b->h_vbeg[q + 1] - b->h_vbeg[q];
  if (run_items == 0 || 2 * run_items > it_nvi(b)) return;
  std::vector<VecItem> vis;
  std::vector<int32_t> vbeg(b->n + 1);
  for (int q = 0; q < b->n; ++q) {
    vbeg[q] = (int32_t)vis.size();
    if (b->host_st[q].done == 0)
      vis.insert(vis.end(), b->h_vis.begin() + b->h_vbeg[q],
                 b->h_vis.begin() + b->h_vbeg[q + 1]);
  }
  vbeg[b->n] = (int32_t)vis.size();
  SEM_HIP(hipMemcpyAsync(b->vitems_c.p, vis.data(), vis.size() * sizeof(VecItem),
                         hipMemcpyHostToDevice, b->s));
  SEM_HIP(hipMemcpyAsync(b->vbeg_c.p, vbeg.data(), vbeg.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, b->s));
  for (int k = 0; k < 3; ++k) {
    std::vector<AxItem> ax;
    for (int q = 0; q < b->n; ++q)
      if (b->host_st[q].done == 0)
        ax.insert(ax.end(), b->h_ax[k].begin() + b->h_axbeg[k][q],
                  b->h_ax[k].begin() + b->h_axbeg[k][q + 1]);
    SEM_HIP(hipMemcpyAsync(b->axitems_c[k].p, ax.data(), ax.size() * sizeof(AxItem),
                           hipMemcpyHostToDevice, b->s));
    b->n_ax_c[k] = (int)ax.size();
  }
  // the host vectors are read by the copies above before they go away
  SEM_HIP(hipStreamSynchronize(b->s));
  b->n_vi_c = (int)vis.size();
  for (auto it = b->graphs.begin(); it != b->graphs.end();)
    if (it->ver != 0) {
      (void)hipGraphExecDestroy(it->exec);
      it = b->graphs.erase(it);
    } else {
      ++it;
    }
  b->list_ver += 1;
  b->compact = true;
}

// Run CG iterations until every solve's flag is set.  Returns true when the
// stagnation monitor stopped solve 0 (its residual norm fell by less than 2x
// over the last >= 200 iterations), which the learned path treats as a
// reason to fall back to Jacobi.
static bool run_cg(sem_batch *b, int prec, int jac, const sem_solve_opts *o,
                   int mode = 0, bool monitor = false, double ref_rate = 0.0) {
  // the other passes over a batch (initialisation, residuals) use the full
  // lists: the compacted ones live for one run of CG iterations
  struct Restore {
    sem_batch *b;
    ~Restore() { b->compact = false; }
  } restore{b};
  const int K = std::max(1, o->check_every);
  std::vector<std::pair<int, double>> hist;  // (iteration, best rr so far)
  double best = 0.0;
  auto poll = [&]() {
    SEM_HIP(hipMemcpyAsync(b->host_st, b->st.p, b->n * sizeof(CgState),
                           hipMemcpyDeviceToHost, b->s));
    SEM_HIP(hipStreamSynchronize(b->s));
    for (int q = 0; q < b->n; ++q)
      if (b->host_st[q].done == 0) return false;
    return true;
  };
  while (!poll()) {
    if (monitor) {
      // The residual 2-norm of flexible CG is not monotone (CG minimises the
      // energy norm), so both guards use the smallest residual so far.
      const CgState &c = b->host_st[0];
      best = hist.empty() ? c.rr : std::min(best, c.rr);
      // progress check: after 300 iterations the learned solve must have
      // reduced log10 ||r|| / ||b|| by at least 30% as much as Jacobi-PCG
      // does on average on this operator (ref_rate, measured on the
      // training solves; CG's own rate is uneven, so the bar is low: it
      // catches a network that stalls the solve, not one that is merely
      // no better than Jacobi)
      if (ref_rate < 0.0 && c.it >= 300 && c.bb > 0.0 && best > 0.0 &&
          0.5 * std::log10(best / c.bb) > 0.3 * ref_rate * c.it)
        return true;
      // stagnation: less than a halving of the best residual over 400
      // iterations
      hist.push_back({c.it, best});
      for (auto it = hist.rbegin(); it != hist.rend(); ++it)
        if (c.it - it->first >= 400) {
          if (best > 0.25 * it->second) return true;
          break;
        }
    }
    if (mode == 0) maybe_compact(b);
    if (o->use_graph)
      SEM_HIP(hipGraphLaunch(get_graph(b, prec, K, jac, mode), b->s));
    else
      for (int q = 0; q < K; ++q) iteration(b, prec, jac, mode);
    if (b->snap_x != nullptr && b->snap_count < b->snap_max) {
      sem_handle *h = b->hs[0];
      const size_t bytes = (size_t)h->nG * sizeof(double);
      SEM_HIP(hipMemcpyAsync(b->snap_x + (size_t)b->snap_count * h->nG,
                             b->hsd[0].v64[VX], bytes, hipMemcpyDeviceToDevice,
                             b->s));
      SEM_HIP(hipMemcpyAsync(b->snap_r + (size_t)b->snap_count * h->nG,
                             b->hsd[0].v64[VR], bytes, hipMemcpyDeviceToDevice,
                             b->s));
      b->snap_count += 1;
    }
  }
  return false;
}

// --------------------------------------------------------------------------
// solve
// --------------------------------------------------------------------------
static void check_opts(const sem_solve_opts *o) {
  if (!(o->rtol > 0.0) || o->maxit < 0 || o->check_every < 1)
    fail(SEM_ERR_ARG, "solve: need rtol > 0, maxit >= 0, check_every >= 1");
  if (o->pc != SEM_PC_NONE && o->pc != SEM_PC_JACOBI && o->pc != SEM_PC_LEARNED)
    fail(SEM_ERR_ARG, "solve: unknown preconditioner");
  if (o->inner_prec != SEM_FP64 && o->inner_prec != SEM_FP32 &&
      o->inner_prec != SEM_BF16 && o->inner_prec != SEM_BF16_PLAIN_D &&
      o->inner_prec != SEM_BF16_MFMA)
    fail(SEM_ERR_ARG, "solve: unknown inner precision");
  if (o->inner_prec != SEM_FP64 && !(o->inner_rtol > 0.0 && o->inner_rtol < 1.0))
    fail(SEM_ERR_ARG, "solve: inner_rtol must be in (0, 1)");
}

sem_status batch_solve(sem_batch *b, const sem_solve_opts *o,
                       const double *const *bL, double *const *xL,
                       sem_solve_stats *stats, hipStream_t caller) {
  check_opts(o);
  for (int q = 0; q < b->n; ++q)
    if (bL[q] == nullptr || xL[q] == nullptr || (const void *)bL[q] == xL[q])
      fail(SEM_ERR_ARG, "solve: null or aliased b / x");
  hipStream_t s = b->s;
  // a batch with its own stream orders it after the caller's work; one laid
  // out in caller memory runs on the caller's stream and is timed on the host
  std::chrono::steady_clock::time_point t0, t1;
  if (b->owned) {
    SEM_HIP(hipEventRecord(b->fence, caller));
    SEM_HIP(hipStreamWaitEvent(s, b->fence, 0));
    SEM_HIP(hipEventRecord(b->ev0, s));
  } else {
    SEM_HIP(hipStreamSynchronize(s));
    t0 = std::chrono::steady_clock::now();
  }
  // the learned preconditioner is Jacobi plus a correction, and falls back
  // to Jacobi
  const int jac = o->pc == SEM_PC_JACOBI || o->pc == SEM_PC_LEARNED;
  const int n = b->n;
  for (int q = 0; q < n; ++q) {
    sem_handle *h = b->hs[q];
    hipLaunchKernelGGL(k_first_copy, dim3(nblk(h->nG)), dim3(RT), 0, s, h->nG,
                       h->offsets.as<int32_t>(), h->perm.as<int32_t>(), bL[q],
                       (double *)b->hsd[q].v64[VB]);
    hipLaunchKernelGGL(k_first_copy, dim3(nblk(h->nG)), dim3(RT), 0, s, h->nG,
                       h->offsets.as<int32_t>(), h->perm.as<int32_t>(), xL[q],
                       (double *)b->hsd[q].v64[VX]);
  }
  SEM_HIP(hipGetLastError());

  std::vector<int> iters(n, 0), outer(n, 0), status(n, SEM_ERR_NOT_CONVERGED);
  std::vector<double> contraction(n, 0.0);
  std::vector<int> act(n, 1), mx(n, o->maxit);
  bool learned = o->pc == SEM_PC_LEARNED;
  int fell_back = 0;
  if (learned) {
    if (n != 1) fail(SEM_ERR_ARG, "solve: the learned preconditioner needs a single solve");
    if (!learn_active(b->hs[0]))
      fail(SEM_ERR_STATE, "solve: no network attached (sem_learn_attach)");
    learn_refresh(b->hs[0]);
    if (learn_damping(b->hs[0]) == 0.0) {
      // validation found no gain over Jacobi: the correction is disabled
      learned = false;
      fell_back = 1;
    }
  }
  if (o->inner_prec == SEM_FP64) {
    upload_active(b, act, mx);
    init(b, SEM_FP64, learned ? 1 : jac, false, o->rtol * o->rtol);
    bool stagnated = false;
    if (learned) {
      init_fcg(b, SEM_FP64);
      stagnated = run_cg(b, SEM_FP64, 1, o, 1, true, learn_ref_rate(b->hs[0]));
    } else {
      run_cg(b, SEM_FP64, jac, o);
    }
    for (int q = 0; q < n; ++q) iters[q] = b->host_st[q].it;
    if (learned && (stagnated || b->host_st[0].done != 1)) {
      // fall back: Jacobi-PCG from the current iterate (x is only updated
      // with finite steps), remaining iteration budget
      fell_back = 1;
      mx[0] = std::max(0, o->maxit - iters[0]);
      upload_active(b, act, mx);
      init(b, SEM_FP64, 1, false, o->rtol * o->rtol);
      run_cg(b, SEM_FP64, 1, o);
      iters[0] += b->host_st[0].it;
    }
    for (int q = 0; q < n; ++q) {
      const int d = b->host_st[q].done;
      status[q] = d == 1 ? SEM_OK : d == 2 ? SEM_ERR_BREAKDOWN : SEM_ERR_NOT_CONVERGED;
    }
  } else {
    // FP64 iterative refinement: r = b - A64 x; the inner solve (PCG, or
    // flexible CG with the learned correction) solves A_lo d = r / ||r|| with
    // FP32 vectors and an FP32 or BF16-stored operator (FP64 dots and
    // scalars); x += ||r|| d.  The FP64 true residual decides every step.
    const int prec = o->inner_prec;
    std::vector<double> rel_prev(n, 1e300);
    std::vector<int> stall(n, 0);
    contraction.assign(n, 0.0);
    upload_active(b, act, mx);
    residual(b);
    while (true) {
      int n_active = 0;
      for (int q = 0; q < n; ++q) {
        if (!act[q]) continue;
        const double rr = b->host_red[2 * q], bb = b->host_red[2 * q + 1];
        if (!std::isfinite(rr)) {
          status[q] = SEM_ERR_BREAKDOWN;
          act[q] = 0;
          continue;
        }
        const double rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        if (rel <= o->rtol) {
          status[q] = SEM_OK;
          act[q] = 0;
          continue;
        }
        if (learned && rel > 0.5 * rel_prev[q]) {
          // the learned step did not halve the true residual: undo it and
          // continue with Jacobi
          hipLaunchKernelGGL(k_baxpy_mixed, dim3(vec_grid(b)), dim3(RT), 0, s,
                             b->sds.as<BatchSolve>(), b->active.as<int32_t>(),
                             b->scale.as<double>(), b->vitems.as<VecItem>(),
                             b->n_vi);  // (scale holds -1/||r_old||)
          SEM_HIP(hipGetLastError());
          learned = false;
          fell_back = 1;
          residual(b);
          q -= 1;  // re-evaluate this solve with the restored iterate
          continue;
        }
        stall[q] = rel > 0.9 * rel_prev[q] ? stall[q] + 1 : 0;
        if (rel_prev[q] < 1e300)
          contraction[q] = std::max(contraction[q], rel / rel_prev[q]);
        rel_prev[q] = rel;
        if (iters[q] >= o->maxit || stall[q] >= 3) {
          act[q] = 0;  // not converged
          continue;
        }
        b->host_d[q] = 1.0 / std::sqrt(rr);
        mx[q] = o->maxit - iters[q];
        ++n_active;
      }
      if (n_active == 0) break;
      SEM_HIP(hipMemcpyAsync(b->scale.p, b->host_d, n * sizeof(double),
                             hipMemcpyHostToDevice, s));
      upload_active(b, act, mx);
      const BatchSolve *sds = b->sds.as<BatchSolve>();
      const VecItem *vi = b->vitems.as<VecItem>();
      const int g = vec_grid(b);
      hipLaunchKernelGGL(k_bscale_cast, dim3(g), dim3(RT), 0, s, sds,
                         b->active.as<int32_t>(), b->scale.as<double>(), vi,
                         b->n_vi);
      SEM_HIP(hipGetLastError());
      bool bad = false;
      if (learned) {
        init(b, prec, 1, true, o->inner_rtol * o->inner_rtol);
        init_fcg(b, prec);
        const bool stag =
            run_cg(b, prec, 1, o, 1, true, learn_ref_rate(b->hs[0]));
        bad = stag || b->host_st[0].done == 2;
        iters[0] += b->host_st[0].it;
        if (bad) {
          // breakdown, NaN or stagnation of the learned inner solve: redo
          // this step with Jacobi
          learned = false;
          fell_back = 1;
        }
      }
      if (!learned && (bad || o->pc != SEM_PC_LEARNED || fell_back)) {
        init(b, prec, jac || o->pc == SEM_PC_LEARNED, true,
             o->inner_rtol * o->inner_rtol);
        run_cg(b, prec, jac || o->pc == SEM_PC_LEARNED, o);
        for (int q = 0; q < n; ++q)
          if (act[q]) iters[q] += b->host_st[q].it;
      }
      for (int q = 0; q < n; ++q) {
        if (!act[q]) continue;
        outer[q] += 1;
        if (b->host_st[q].done == 2) {
          status[q] = SEM_ERR_BREAKDOWN;
          act[q] = 0;
        }
      }
      upload_active(b, act, mx);
      hipLaunchKernelGGL(k_baxpy_mixed, dim3(g), dim3(RT), 0, s, sds,
                         b->active.as<int32_t>(), b->scale.as<double>(), vi,
                         b->n_vi);
      SEM_HIP(hipGetLastError());
      if (learned) {
        // keep -1/||r|| so that a rejected step can be undone
        for (int q = 0; q < n; ++q) b->host_d[q] = -b->host_d[q];
        SEM_HIP(hipMemcpyAsync(b->scale.p, b->host_d, n * sizeof(double),
                               hipMemcpyHostToDevice, s));
      }
      residual(b);
    }
  }
  for (int q = 0; q < n; ++q) {
    sem_handle *h = b->hs[q];
    hipLaunchKernelGGL(k_scatter, dim3(nblk(h->nL)), dim3(RT), 0, s, h->nL,
                       h->l2g.as<int32_t>(), (const double *)b->hsd[q].v64[VX],
                       xL[q]);
  }
  SEM_HIP(hipGetLastError());
  if (b->owned) {
    SEM_HIP(hipEventRecord(b->ev1, s));
  } else {
    SEM_HIP(hipStreamSynchronize(s));
    t1 = std::chrono::steady_clock::now();
  }
  // recomputed FP64 residuals of every solve
  std::vector<int> all(n, 1);
  upload_active(b, all, mx);
  residual(b);
  float ms = 0.0f;
  if (b->owned)
    SEM_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  else
    ms = (float)std::chrono::duration<double, std::milli>(t1 - t0).count();
  sem_status worst = SEM_OK;
  for (int q = 0; q < n; ++q) {
    if (stats != nullptr) {
      const double rr = b->host_red[2 * q], bb = b->host_red[2 * q + 1];
      stats[q].iters = iters[q];
      stats[q].outer_iters = outer[q];
      stats[q].status = status[q];
      stats[q].fell_back = fell_back;
      stats[q].final_rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
      stats[q].seconds = ms * 1e-3;
      stats[q].outer_contraction = contraction[q];
    }
    if (status[q] != SEM_OK && worst == SEM_OK) worst = (sem_status)status[q];
  }
  if (b->owned) {
    SEM_HIP(hipEventRecord(b->fence, s));
    SEM_HIP(hipStreamWaitEvent(caller, b->fence, 0));
  }
  return worst;
}

sem_status pcg_solve(sem_handle *h, const sem_solve_opts *o, const double *b_L,
                     double *x_L, sem_solve_stats *st, hipStream_t caller) {
  check_opts(o);
  ensure_vectors(h);
  if (h->ws->single == nullptr) {
    sem_handle *one[1] = {h};
    h->ws->single = batch_create(one, 1);
  }
  const double *bl[1] = {b_L};
  double *xl[1] = {x_L};
  return batch_solve(h->ws->single, o, bl, xl, st, caller);
}

// --------------------------------------------------------------------------
// solve without allocation: every device buffer of a plain FP64 PCG solve
// (solver vectors, descriptor, work lists, partial sums, scalars) is carved
// from one file-scope array that each GPU holds for the life of the process.
// Nothing in it has to start at zero: every buffer is written before it is
// read (the descriptor and work lists are uploaded, the rest is written by
// the initialisation kernels).  Calls that overlap in time on one GPU share
// the array and race.
// --------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES];  // that GPU's copy, or null

// device address of the current GPU's copy of `scratch` (the host-side name
// is not a device address)
static unsigned char *scratch_address() {
  int dev = 0;
  SEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    fail(SEM_ERR_ARG, "solve_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    SEM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr) fail(SEM_ERR_HIP, "solve_noalloc: no address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

size_t noalloc_bytes(const sem_handle *h) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t nG = (size_t)h->nG, nL = (size_t)h->nL, nvi = (nG + VCH - 1) / VCH;
  return (NVEC - 1) * up(nG * 8) + up(nL * 8) + up(nG * 8) + up((size_t)h->E * 8) +
         up(sizeof(BatchSolve)) + up(sizeof(CgState)) + up(nvi * sizeof(VecItem)) +
         up(2 * sizeof(int32_t)) + up(3 * nvi * 8) + up(2 * 8) + 3 * up(8);
}

sem_status pcg_solve_noalloc(sem_handle *h, const sem_solve_opts *o,
                             const double *b_L, double *x_L, sem_solve_stats *st,
                             hipStream_t caller) {
  check_opts(o);
  if (o->inner_prec != SEM_FP64 || o->pc == SEM_PC_LEARNED)
    fail(SEM_ERR_ARG, "solve_noalloc: plain FP64 PCG only (inner_prec SEM_FP64, "
                      "preconditioner none or Jacobi)");
  const size_t need_bytes = noalloc_bytes(h);
  if (need_bytes > SCRATCH_BYTES)
    fail(SEM_ERR_ARG, "solve_noalloc: the mesh needs " + std::to_string(need_bytes) +
                          " bytes of solver memory, more than the 33554432 available");
  unsigned char *base = scratch_address();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void *p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  sem_batch b;
  b.owned = false;
  b.hs.assign(1, h);
  b.n = 1;
  b.nset = h->n1;
  b.orders.assign(1, h->n1);
  void *v64[NVEC], *v32[NVEC];
  for (int v = 0; v < NVEC; ++v) {
    v64[v] = take((size_t)(v == VWL ? h->nL : h->nG) * 8);
    v32[v] = nullptr;
  }
  double *one64 = (double *)take((size_t)h->nG * 8);
  double *edot = (double *)take((size_t)h->E * 8);
  b.hsd.assign(1, describe(h, 0, v64, v32, one64, nullptr, edot));
  b.periodic = h->periodic != 0;
  b.wide = h->nL > (int64_t)UINT32_MAX;
  b.sum_nG = h->nG;
  b.sum_nL = h->nL;
  std::vector<VecItem> vis;
  for (int64_t g = 0; g < h->nG; g += VCH) vis.push_back({0, 0, g});
  b.n_vi = (int)vis.size();
  const int32_t vbeg[2] = {0, b.n_vi};
  b.sds.view(take(sizeof(BatchSolve)), sizeof(BatchSolve));
  b.st.view(take(sizeof(CgState)), sizeof(CgState));
  b.vitems.view(take(vis.size() * sizeof(VecItem)), vis.size() * sizeof(VecItem));
  b.vbeg.view(take(sizeof vbeg), sizeof vbeg);
  b.part.view(take(3 * vis.size() * 8), 3 * vis.size() * 8);
  b.red.view(take(2 * 8), 2 * 8);
  b.active.view(take(8), sizeof(int32_t));
  b.maxit.view(take(8), sizeof(int32_t));
  b.scale.view(take(8), sizeof(double));
  if (off != need_bytes) fail(SEM_ERR_STATE, "solve_noalloc: scratch layout mismatch");
  b.host_st = b.inl_st;
  b.host_red = b.inl_red;
  b.host_i = b.inl_i;
  b.host_d = b.inl_d;
  b.s = caller;
  SEM_HIP(hipMemcpyAsync(b.sds.p, b.hsd.data(), sizeof(BatchSolve),
                         hipMemcpyHostToDevice, caller));
  SEM_HIP(hipMemcpyAsync(b.vitems.p, vis.data(), vis.size() * sizeof(VecItem),
                         hipMemcpyHostToDevice, caller));
  SEM_HIP(hipMemcpyAsync(b.vbeg.p, vbeg, sizeof vbeg, hipMemcpyHostToDevice, caller));
  hipLaunchKernelGGL(k_unmask, dim3(nblk(h->nG)), dim3(RT), 0, caller, h->nG,
                     h->gmask.as<uint8_t>(), one64, (float *)nullptr);
  SEM_HIP(hipGetLastError());
  SEM_HIP(hipStreamSynchronize(caller));  // the host sources of the uploads
  sem_solve_opts oo = *o;
  oo.use_graph = 0;  // kernels are launched directly
  const double *bl[1] = {b_L};
  double *xl[1] = {x_L};
  return batch_solve(&b, &oo, bl, xl, st, caller);
}

// FP64 Jacobi-PCG from x_L with snapshots of (x_k, r_k) every `every`
// iterations (at most max_snaps); returns the number recorded.  The
// converged solution stays in the handle's FP64 x vector.
int solve_with_snapshots(sem_handle *h, const double *bL, double *xL, double rtol,
                         int every, int max_snaps, double *xs, double *rs,
                         int *iters, hipStream_t caller) {
  ensure_vectors(h);
  if (h->ws->single == nullptr) {
    sem_handle *one[1] = {h};
    h->ws->single = batch_create(one, 1);
  }
  sem_batch *b = h->ws->single;
  sem_solve_opts o{};
  o.rtol = rtol;
  o.maxit = 1000000;
  o.pc = SEM_PC_JACOBI;
  o.inner_prec = SEM_FP64;
  o.inner_rtol = 0.1;
  o.check_every = every;
  o.use_graph = 1;
  b->snap_x = xs;
  b->snap_r = rs;
  b->snap_max = max_snaps;
  b->snap_count = 0;
  const double *bl[1] = {bL};
  double *xl[1] = {xL};
  sem_status st;
  sem_solve_stats ss{};
  try {
    st = batch_solve(b, &o, bl, xl, &ss, caller);
  } catch (...) {
    b->snap_x = b->snap_r = nullptr;
    throw;
  }
  const int n = b->snap_count;
  if (iters) *iters = ss.iters;
  b->snap_x = b->snap_r = nullptr;
  b->snap_max = b->snap_count = 0;
  if (st != SEM_OK) fail(st, "train: the FP64 data solve did not converge");
  return n;
}

const double *solution_vector(sem_handle *h) { return h->ws->v64[VX].as<double>(); }

// captured graphs hold the buffers of the network attached when they were
// captured: drop them whenever the attachment changes
void drop_graphs(sem_handle *h) {
  if (h->ws == nullptr || h->ws->single == nullptr) return;
  sem_batch *b = h->ws->single;
  SEM_HIP(hipStreamSynchronize(b->s));
  for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

// --------------------------------------------------------------------------
// autotuner: time the batched operator for each block size and persistent
// grid, keep the fastest per precision; results cached in a JSON file named
// by the SEM_AUTOTUNE_CACHE environment variable (if set)
// --------------------------------------------------------------------------
static std::string tune_key(const sem_batch *b, int prec) {
  int64_t nodes = 0;
  for (auto *h : b->hs) nodes += h->nL;
  int bucket = 0;
  while ((int64_t)1 << (bucket + 1) <= nodes) ++bucket;
  hipDeviceProp_t p;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&p, dev);
  std::ostringstream k;
  k << p.gcnArchName << "|set" << b->nset << "|prec" << prec << "|log2nodes"
    << bucket;
  std::string s = k.str();
  for (auto &c : s)
    if (c == '"' || c == '\\' || c == ':') c = '_';
  return s;
}

static std::map<std::string, std::pair<int, int>> read_cache(const char *path) {
  std::map<std::string, std::pair<int, int>> m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    // one entry per line: "key": [bs, gmul],
    const size_t a = line.find('"'), b2 = line.find('"', a + 1);
    const size_t l = line.find('['), c = line.find(',', l), r = line.find(']', l);
    if (a == std::string::npos || b2 == std::string::npos ||
        l == std::string::npos || c == std::string::npos || r == std::string::npos)
      continue;
    const int bs = atoi(line.substr(l + 1, c - l - 1).c_str());
    const int gm = atoi(line.substr(c + 1, r - c - 1).c_str());
    if (bs == 64 || bs == 128 || bs == 256) m[line.substr(a + 1, b2 - a - 1)] = {bs, gm};
  }
  return m;
}

static void write_cache(const char *path,
                        const std::map<std::string, std::pair<int, int>> &m) {
  std::ofstream f(std::string(path) + ".tmp");
  f << "{\n";
  size_t q = 0;
  for (auto &kv : m) {
    f << "  \"" << kv.first << "\": [" << kv.second.first << ", "
      << kv.second.second << "]" << (++q < m.size() ? "," : "") << "\n";
  }
  f << "}\n";
  f.close();
  std::rename((std::string(path) + ".tmp").c_str(), path);
}

void batch_tune(sem_batch *b, int prec, int *best_bs, int *best_gm,
                double *best_us) {
  if (prec < SEM_FP64 || prec > SEM_BF16)
    fail(SEM_ERR_ARG, "tune: precision must be SEM_FP64, SEM_FP32 or SEM_BF16");
  const char *path = getenv("SEM_AUTOTUNE_CACHE");
  const std::string key = tune_key(b, prec);
  if (path) {
    auto m = read_cache(path);
    auto it = m.find(key);
    // an entry whose block cannot hold an element of this set is ignored
    if (it != m.end() && it->second.first >= bax_min_block(b->nset)) {
      b->bs[prec] = it->second.first;
      b->gmul[prec] = it->second.second;
      if (best_bs) *best_bs = b->bs[prec];
      if (best_gm) *best_gm = b->gmul[prec];
      if (best_us) *best_us = -1.0;
      return;
    }
  }
  // operator input: the p vectors hold whatever they hold; timing only
  std::vector<int> all(b->n, 1), mx(b->n, 1);
  upload_active(b, all, mx);
  const int bss[3] = {64, 128, 256};
  const int gms[5] = {0, 4, 8, 16, 32};
  double best = 1e300;
  int bbs = b->bs[prec], bgm = b->gmul[prec];
  for (int bs : bss) {
    if (bs < bax_min_block(b->nset)) continue;  // cannot hold an element
    for (int gm : gms) {
      b->bs[prec] = bs;
      b->gmul[prec] = gm;
      bax(b, prec, VP, VWL, 0);  // warm
      SEM_HIP(hipEventRecord(b->ev0, b->s));
      const int reps = 3;
      for (int r = 0; r < reps; ++r) bax(b, prec, VP, VWL, 0);
      SEM_HIP(hipEventRecord(b->ev1, b->s));
      SEM_HIP(hipEventSynchronize(b->ev1));
      float ms = 0;
      SEM_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
      const double us = ms * 1e3 / reps;
      if (us < best) {
        best = us;
        bbs = bs;
        bgm = gm;
      }
    }
  }
  b->bs[prec] = bbs;
  b->gmul[prec] = bgm;
  for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
  if (path) {
    auto m = read_cache(path);
    m[key] = {bbs, bgm};
    write_cache(path, m);
  }
  if (best_bs) *best_bs = bbs;
  if (best_gm) *best_gm = bgm;
  if (best_us) *best_us = best;
}

}  // namespace sem
