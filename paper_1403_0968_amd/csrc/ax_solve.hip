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
// a mass term passes H = alpha(X) B and the kernel adds H o u.
#include "ax_tile.h"

namespace sem {

template <int N1, class TV, class TG, class TC, bool MASS>
__global__ void __launch_bounds__((OpShape<N1, sizeof(TC)>::THREADS))
    k_ax_solve(int64_t E, const TC *__restrict__ D, const TG *__restrict__ G,
               const TV *__restrict__ u, TV *__restrict__ w, Box box,
               const int32_t *__restrict__ stop, const TG *__restrict__ H) {
  using S = OpShape<N1, sizeof(TC)>;
  __shared__ TC smem[lds_words<N1>(S::EPB)];
  if (stop != nullptr && *stop != 0) return;  // uniform: the solve finished
  ax_tile<N1, S::EPB, TV, TG, TV, TC, true, false, MASS, S::NTG>(
      threadIdx.x, (int64_t)blockIdx.x * S::EPB, E, D, G, u, w, &box, smem, H);
}

template <int N1, class TV, class TG, class TC>
static void launch_solve_t(int64_t E, const void *D, const void *G,
                           const void *H, const void *u, void *w, const Box &box,
                           const int32_t *stop, hipStream_t s) {
  using S = OpShape<N1, sizeof(TC)>;
  const int64_t blocks = (E + S::EPB - 1) / S::EPB;
  if (blocks == 0) return;
  const dim3 grid((unsigned)blocks), block(S::THREADS);
  if (H != nullptr)
    hipLaunchKernelGGL((k_ax_solve<N1, TV, TG, TC, true>), grid, block, 0, s, E,
                       (const TC *)D, (const TG *)G, (const TV *)u, (TV *)w, box,
                       stop, (const TG *)H);
  else
    hipLaunchKernelGGL((k_ax_solve<N1, TV, TG, TC, false>), grid, block, 0, s, E,
                       (const TC *)D, (const TG *)G, (const TV *)u, (TV *)w, box,
                       stop, (const TG *)nullptr);
}

template <int N1>
static void launch_solve_n(int prec, int64_t E, const void *D, const void *G,
                           const void *H, const void *u, void *w, const Box &box,
                           const int32_t *stop, hipStream_t s) {
  if (prec == SEM_FP64)
    launch_solve_t<N1, double, double, double>(E, D, G, H, u, w, box, stop, s);
  else if (prec == SEM_FP32)
    launch_solve_t<N1, float, float, float>(E, D, G, H, u, w, box, stop, s);
  else
    launch_solve_t<N1, float, uint16_t, float>(E, D, G, H, u, w, box, stop, s);
}

void launch_ax_solve(int N, int prec, int64_t E, const void *D, const void *G,
                     const void *H, const void *u, void *w, const Box &box,
                     const int32_t *stop, hipStream_t s) {
  switch (N) {
    case 1: launch_solve_n<2>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 2: launch_solve_n<3>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 3: launch_solve_n<4>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 4: launch_solve_n<5>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 5: launch_solve_n<6>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 6: launch_solve_n<7>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 7: launch_solve_n<8>(prec, E, D, G, H, u, w, box, stop, s); break;
    case 8: launch_solve_n<9>(prec, E, D, G, H, u, w, box, stop, s); break;
    default: fail(SEM_ERR_ARG, "solve: N must be in 1..8");
  }
  SEM_HIP(hipGetLastError());
}

}  // namespace sem
