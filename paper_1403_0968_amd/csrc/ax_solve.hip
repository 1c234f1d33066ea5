// The gathered operator of a single solve, w_L = A_L Q p_G (paper section
// 4.2.1 operator, applied inside the PCG of section 4.2.2): the element
// routine of the standalone operator with GATHER on, every pointer, the
// closed-form box numbering and the solver's done flag passed as kernel
// arguments.  A workgroup then issues its data loads at once; the batched
// kernel first has to fetch its work item and the solve's descriptor, a
// chain of dependent loads that cost ~25 % of the operator time at 32^3,
// N = 7 (measured with and without the gather: the gather itself costs
// nothing in FP64).  Workgroup shapes and load hints as the standalone
// operator (OpShape).  A mesh with
// a mass term passes H = alpha(X) B and the kernel adds H o u.  With edot
// non-null the kernel also stores every element's energy p_e^T w_e (the
// element terms of (p, A p), in an order fixed by the node indices).
// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD
// b % 8), each with its own L2.  With FP32 / BF16 storage the kernel numbers
// its element blocks so that every XCD gets one contiguous run of them, and
// elements that share nodes of the gathered vector (neighbours along x, y
// and z) read the shared cache lines through the same L2: 102 -> 94 us at
// 32^3, N = 7, FP32.  In FP64 the same order was slower (181 -> 186 us), so
// FP64 keeps the plain order.  NTW (a solve whose vectors exceed the
// last-level cache): the output is stored non-temporally, as in the
// standalone operator: 188 -> 182 us FP64 at 32^3, N = 7, and the assembly
// that reads it next got faster too (FP32 56 -> 52 us).
#include "ax_tile.h"

namespace sem {

// element block of workgroup b of nb: XCD x = b % 8 takes the run
// [x q + min(x, r), ...) of q or q + 1 blocks (q = nb / 8, r = nb % 8)
__device__ inline int64_t xcd_run_block(unsigned b, unsigned nb) {
  const unsigned q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
  return (int64_t)x * q + (x < r ? x : r) + k;
}

template <int N1, class TV, class TG, class TC, bool MASS, bool EDOT, bool NTW>
__global__ void __launch_bounds__((OpShape<N1, sizeof(TC)>::THREADS))
    k_ax_solve(int64_t E, const TC *__restrict__ D, const TG *__restrict__ G,
               const TV *__restrict__ u, TV *__restrict__ w, Box box,
               const int32_t *__restrict__ stop, const TG *__restrict__ H,
               double *__restrict__ edot) {
  using S = OpShape<N1, sizeof(TC)>;
  __shared__ __align__(16) TC smem[lds_words<N1, TC>(S::EPB)];
  // the done flag of the solve is checked inside, after the loads are issued
  ax_tile<N1, S::EPB, TV, TG, TV, TC, true, NTW, MASS, S::NTG, EDOT, S::PRED>(
      threadIdx.x,
      (sizeof(TV) == 4 ? xcd_run_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x) *
          S::EPB,
      E, D, G, u, w, &box, smem, H, edot, stop);
}

template <int N1, class TV, class TG, class TC, bool MASS, bool NTW>
static void launch_solve_w(int64_t E, const void *D, const void *G,
                           const void *H, const void *u, void *w, const Box &box,
                           const int32_t *stop, double *edot, hipStream_t s) {
  using S = OpShape<N1, sizeof(TC)>;
  const int64_t blocks = (E + S::EPB - 1) / S::EPB;
  if (blocks == 0) return;
  const dim3 grid((unsigned)blocks), block(S::THREADS);
  if (edot != nullptr)
    hipLaunchKernelGGL((k_ax_solve<N1, TV, TG, TC, MASS, true, NTW>), grid, block, 0, s,
                       E, (const TC *)D, (const TG *)G, (const TV *)u, (TV *)w,
                       box, stop, (const TG *)H, edot);
  else
    hipLaunchKernelGGL((k_ax_solve<N1, TV, TG, TC, MASS, false, NTW>), grid, block, 0,
                       s, E, (const TC *)D, (const TG *)G, (const TV *)u, (TV *)w,
                       box, stop, (const TG *)H, edot);
}

template <int N1, class TV, class TG, class TC, bool MASS>
static void launch_solve_m(int64_t E, const void *D, const void *G,
                           const void *H, const void *u, void *w, const Box &box,
                           const int32_t *stop, double *edot, bool nt, hipStream_t s) {
  if (nt)
    launch_solve_w<N1, TV, TG, TC, MASS, true>(E, D, G, H, u, w, box, stop, edot, s);
  else
    launch_solve_w<N1, TV, TG, TC, MASS, false>(E, D, G, H, u, w, box, stop, edot, s);
}

template <int N1, class TV, class TG, class TC>
static void launch_solve_t(int64_t E, const void *D, const void *G,
                           const void *H, const void *u, void *w, const Box &box,
                           const int32_t *stop, double *edot, bool nt, hipStream_t s) {
  if (H != nullptr)
    launch_solve_m<N1, TV, TG, TC, true>(E, D, G, H, u, w, box, stop, edot, nt, s);
  else
    launch_solve_m<N1, TV, TG, TC, false>(E, D, G, H, u, w, box, stop, edot, nt, s);
}

template <int N1>
static void launch_solve_n(int prec, int64_t E, const void *D, const void *G,
                           const void *H, const void *u, void *w, const Box &box,
                           const int32_t *stop, double *edot, bool nt, hipStream_t s) {
  if (prec == SEM_FP64)
    launch_solve_t<N1, double, double, double>(E, D, G, H, u, w, box, stop, edot, nt, s);
  else if (prec == SEM_FP32)
    launch_solve_t<N1, float, float, float>(E, D, G, H, u, w, box, stop, edot, nt, s);
  else
    launch_solve_t<N1, float, uint16_t, float>(E, D, G, H, u, w, box, stop, edot, nt, s);
}

void launch_ax_solve(int N, int prec, int64_t E, const void *D, const void *G,
                     const void *H, const void *u, void *w, const Box &box,
                     const int32_t *stop, double *edot, bool nt, hipStream_t s) {
  switch (N) {
    case 1: launch_solve_n<2>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 2: launch_solve_n<3>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 3: launch_solve_n<4>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 4: launch_solve_n<5>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 5: launch_solve_n<6>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 6: launch_solve_n<7>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 7: launch_solve_n<8>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    case 8: launch_solve_n<9>(prec, E, D, G, H, u, w, box, stop, edot, nt, s); break;
    default: fail(SEM_ERR_ARG, "solve: N must be in 1..8");
  }
  SEM_HIP(hipGetLastError());
}

}  // namespace sem
