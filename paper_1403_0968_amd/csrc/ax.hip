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
//   * all loads of an element (its u column and the 6 n1 geometric factors of
//     the column) are issued before any arithmetic, so each wave keeps its
//     whole input in flight; the factors are read once per operator
//     application and bypass the caches (non-temporal loads), and so do the
//     outputs of the standalone operator;
//   * u, the r-flux and the s-flux each have their own LDS array.
// Storage/compute type combinations:
//   FP64: u, G, w double; FP32: float everywhere;
//   BF16: u and G bfloat16, D, arithmetic and w in FP32.  At n1 = 8 the BF16
//   factors are stored column-contiguous ([E][6][n1^2][n1]) so that a lane
//   fetches the 8 values of one factor with a single 16-byte load, and the
//   BF16 input is read in 16-byte rows and redistributed through LDS.
// GATHER = true reads u from a unique-node vector (the Q of the assembled
// operator), used inside the solvers; the unique index of each node comes
// from the closed-form box numbering, so the gather adds no index traffic
// and its loads issue with the others.  With a mass term (alpha != 0) the
// standalone operator also streams H = alpha(X) B and adds H o u (the lumped
// mass operator of equation semOperator): 72 B per node in FP64.
//
// Two kernels share one element routine: k_ax (one tile of elements per
// workgroup, the standalone operator) and k_bax (persistent workgroups
// walking a list of (solve, element tile) items of a batch of independent
// solves with mixed orders; one launch applies the operators of all solves,
// and stores every element's energy p_e^T w_e for the solvers' (p, A p)).
#include "ax_tile.h"

namespace sem {

// ---------------------------------------------------------------------------
// standalone operator: one tile per workgroup
// ---------------------------------------------------------------------------
template <int N1, class TU, class TG, class TW, class TC, bool GATHER, bool NTW,
          bool MASS>
__global__ void __launch_bounds__((OpShape<N1, sizeof(TC)>::THREADS))
    k_ax(int64_t E, const TC *__restrict__ D, const TG *__restrict__ G,
         const TU *__restrict__ u, TW *__restrict__ w,
         const Box *__restrict__ box, const int32_t *__restrict__ stop,
         const TG *__restrict__ H) {
  using S = OpShape<N1, sizeof(TC)>;
  __shared__ __align__(16) TC smem[lds_words<N1, TC>(S::EPB)];
  if (stop != nullptr && *stop != 0) return;  // uniform: solver finished
  ax_tile<N1, S::EPB, TU, TG, TW, TC, GATHER, NTW, MASS, S::NTG, false, S::PRED>(
      threadIdx.x, (int64_t)blockIdx.x * S::EPB, E, D, G, u, w, box, smem, H);
}

template <int N1, class TU, class TG, class TW, class TC>
static void launch_nt(int64_t E, const void *D, const void *G, const void *H,
                      const void *u, void *w, hipStream_t s) {
  using S = OpShape<N1, sizeof(TC)>;
  const int64_t blocks = (E + S::EPB - 1) / S::EPB;
  if (blocks == 0) return;
  const dim3 grid((unsigned)blocks), block(S::THREADS);
  if (H != nullptr)
    hipLaunchKernelGGL((k_ax<N1, TU, TG, TW, TC, false, true, true>), grid, block,
                       0, s, E, (const TC *)D, (const TG *)G, (const TU *)u,
                       (TW *)w, (const Box *)nullptr, (const int32_t *)nullptr,
                       (const TG *)H);
  else
    hipLaunchKernelGGL((k_ax<N1, TU, TG, TW, TC, false, true, false>), grid,
                       block, 0, s, E, (const TC *)D, (const TG *)G,
                       (const TU *)u, (TW *)w, (const Box *)nullptr,
                       (const int32_t *)nullptr, (const TG *)nullptr);
}

template <int N1>
static void launch_n(int prec, int64_t E, const void *D, const void *G,
                     const void *H, const void *u, void *w, hipStream_t s) {
  if (prec == SEM_FP64)
    launch_nt<N1, double, double, double, double>(E, D, G, H, u, w, s);
  else if (prec == SEM_FP32)
    launch_nt<N1, float, float, float, float>(E, D, G, H, u, w, s);
  else
    launch_nt<N1, uint16_t, uint16_t, float, float>(E, D, G, H, u, w, s);
}

void launch_ax(int N, int prec, int64_t E, const void *D, const void *G,
               const void *H, const void *u, void *w, hipStream_t s) {
  switch (N) {
    case 1: launch_n<2>(prec, E, D, G, H, u, w, s); break;
    case 2: launch_n<3>(prec, E, D, G, H, u, w, s); break;
    case 3: launch_n<4>(prec, E, D, G, H, u, w, s); break;
    case 4: launch_n<5>(prec, E, D, G, H, u, w, s); break;
    case 5: launch_n<6>(prec, E, D, G, H, u, w, s); break;
    case 6: launch_n<7>(prec, E, D, G, H, u, w, s); break;
    case 7: launch_n<8>(prec, E, D, G, H, u, w, s); break;
    case 8: launch_n<9>(prec, E, D, G, H, u, w, s); break;
    default: fail(SEM_ERR_ARG, "sem_ax: N must be in 1..8");
  }
  SEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// persistent batched operator: work items are (solve, first element) tiles;
// each workgroup walks items blockIdx.x, blockIdx.x + gridDim.x, ...
// ---------------------------------------------------------------------------
// elements per tile; launches with BS < N1^2 are refused (bax_min_block)
template <int BS, int N1> struct BTile {
  static constexpr int EPB = (BS / (N1 * N1)) > 0 ? BS / (N1 * N1) : 1;
};

template <int BS, class TV, class TG, class TC, int N1>
__device__ __forceinline__ void bax_one(const BatchSolve &sd, int64_t e0,
                                        int src, int dst, TC *smem) {
  const TV *u = (const TV *)(sizeof(TV) == 8 ? sd.v64[src] : sd.v32[src]);
  TV *w = (TV *)(sizeof(TV) == 8 ? sd.v64[dst] : sd.v32[dst]);
  const TG *G = (const TG *)(sizeof(TG) == 8   ? sd.G64
                             : sizeof(TG) == 4 ? sd.G32
                                               : sd.G16);
  const TC *D = (const TC *)(sizeof(TC) == 8 ? sd.D64 : sd.D32);
  // the element energies (p, A p) terms are stored with every application;
  // the output streams non-temporally (a batch's E-vectors together are far
  // larger than the caches: 256 solves 6.98 -> 6.85 s)
  ax_tile<N1, BTile<BS, N1>::EPB, TV, TG, TV, TC, true, true, false, true, true>(
      threadIdx.x, e0, sd.E, D, G, u, w, &sd.box, smem, nullptr, sd.edot);
}

template <int BS, class TV, class TG, class TC, int... N1s>
__global__ void __launch_bounds__(BS)
    k_bax(const BatchSolve *__restrict__ sds, const CgState *__restrict__ st,
          const AxItem *__restrict__ items, int nitems, int src, int dst,
          int skip_done) {
  extern __shared__ __align__(16) unsigned char dyn_smem[];
  TC *smem = reinterpret_cast<TC *>(dyn_smem);
  for (int q = blockIdx.x; q < nitems; q += gridDim.x) {
    const AxItem it = items[q];
    if (skip_done && st[it.solve].done != 0) continue;  // uniform per block
    const BatchSolve &sd = sds[it.solve];
    const int n1 = sd.N1;
    // exactly one of the compiled orders matches the item's order
    ((n1 == N1s ? bax_one<BS, TV, TG, TC, N1s>(sd, it.elem0, src, dst, smem)
                : void()),
     ...);
    __syncthreads();  // the next item may use another LDS layout
  }
}

template <int BS, class TC, int... N1s> constexpr int max_lds_words() {
  int m = 0;
  ((m = lds_words<N1s, TC>(BTile<BS, N1s>::EPB) > m
            ? lds_words<N1s, TC>(BTile<BS, N1s>::EPB)
            : m),
   ...);
  return m;
}

template <int BS, class TV, class TG, class TC, int... N1s>
static void launch_bax_set(const BatchSolve *sds, const CgState *st,
                           const AxItem *items, int nitems, int grid, int src,
                           int dst, int skip_done, hipStream_t s) {
  const size_t lds = (size_t)max_lds_words<BS, TC, N1s...>() * sizeof(TC);
  hipLaunchKernelGGL((k_bax<BS, TV, TG, TC, N1s...>), dim3(grid), dim3(BS), lds,
                     s, sds, st, items, nitems, src, dst, skip_done);
}

template <int BS, class TV, class TG, class TC>
static void launch_bax_bs(int nset, const BatchSolve *sds, const CgState *st,
                          const AxItem *items, int nitems, int grid, int src,
                          int dst, int skip_done, hipStream_t s) {
  // a thread owns one (i, j) column: a workgroup must hold every column of
  // the largest order of the set
  if (BS < bax_min_block(nset))
    fail(SEM_ERR_ARG, "batched operator: block size below n1^2 of an order");
  // order sets compiled: one order (n1 = 2..9) or the mixed set {4, 6, 8}
  switch (nset) {
    case 2: launch_bax_set<BS, TV, TG, TC, 2>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 3: launch_bax_set<BS, TV, TG, TC, 3>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 4: launch_bax_set<BS, TV, TG, TC, 4>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 5: launch_bax_set<BS, TV, TG, TC, 5>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 6: launch_bax_set<BS, TV, TG, TC, 6>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 7: launch_bax_set<BS, TV, TG, TC, 7>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 8: launch_bax_set<BS, TV, TG, TC, 8>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 9: launch_bax_set<BS, TV, TG, TC, 9>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case AX_SET_468: launch_bax_set<BS, TV, TG, TC, 4, 6, 8>(sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    default: fail(SEM_ERR_ARG, "batched operator: unsupported set of orders");
  }
}

template <class TV, class TG, class TC>
static void launch_bax_t(int bs, int nset, const BatchSolve *sds,
                         const CgState *st, const AxItem *items, int nitems,
                         int grid, int src, int dst, int skip_done,
                         hipStream_t s) {
  switch (bs) {
    case 64: launch_bax_bs<64, TV, TG, TC>(nset, sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 128: launch_bax_bs<128, TV, TG, TC>(nset, sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    case 256: launch_bax_bs<256, TV, TG, TC>(nset, sds, st, items, nitems, grid, src, dst, skip_done, s); break;
    default: fail(SEM_ERR_ARG, "batched operator: block size must be 64, 128 or 256");
  }
}

void launch_bax(int prec, int bs, int nset, const BatchSolve *sds,
                const CgState *st, const AxItem *items, int nitems, int grid,
                int src, int dst, int skip_done, hipStream_t s) {
  if (nitems <= 0) return;
  if (prec == SEM_FP64)
    launch_bax_t<double, double, double>(bs, nset, sds, st, items, nitems, grid,
                                         src, dst, skip_done, s);
  else if (prec == SEM_FP32)
    launch_bax_t<float, float, float>(bs, nset, sds, st, items, nitems, grid, src,
                                      dst, skip_done, s);
  else
    launch_bax_t<float, uint16_t, float>(bs, nset, sds, st, items, nitems, grid,
                                         src, dst, skip_done, s);
  SEM_HIP(hipGetLastError());
}

int bax_min_block(int nset) {
  const int n1 = nset == AX_SET_468 ? 8 : nset;
  const int np = n1 * n1;
  return np <= 64 ? 64 : np <= 128 ? 128 : 256;
}

int bax_elements_per_tile(int bs, int n1) {
  const int np = n1 * n1;
  return bs / np > 0 ? bs / np : 1;
}

}  // namespace sem
