// Finite-difference time step of the 2D acoustic wave equation u_tt = u_xx +
// u_yy (paper section 4.1): periodic nx x ny grid, node (i, j) at j nx + i,
// leapfrog in time, a central stencil of 2r + 1 nodes and order 2r per
// direction in space:
//   u_next = 2 u_cur - u_prev + c sum_{k=-r..r} w_k (u_cur(i+k, j) + u_cur(i, j+k)),
// c = dt^2 / dx^2, w the unit-spacing second-derivative weights.
//
// The paper's kernel reads its 4r + 1 neighbours straight from memory, one
// node per work-item.  HBM-bound on MI355X (24 bytes per node: u_cur and
// u_prev read, u_next written), the kernel here reads every value once:
//   * a workgroup owns a strip of FD_TX columns (one thread per column) and a
//     chunk of rows, and marches down the chunk FD_P rows at a time;
//   * each thread keeps the 2r + FD_P values of its column that the
//     y-stencil of the current rows needs in registers (a sliding window:
//     each new row is one load);
//   * the x-stencil reads the current rows from LDS, staged from the
//     registers with r halo columns on each side (double-buffered: one
//     barrier per FD_P rows);
//   * the loads of the next FD_P rows are issued before the current rows are
//     computed, so every wave keeps loads in flight across the barrier;
//   * short row chunks (16 rows for r <= 2, 32 otherwise; timed on 8192^2)
//     give many workgroups, which a stream of two reads and one write needs
//     to approach the bandwidth a plain copy reaches (a flat
//     2-read-1-write kernel reaches 75 % of peak here), at the price of
//     re-reading 2r rows per chunk from cache;
//   * blocks are numbered row-major over (strip, chunk): workgroups are
//     dealt to the 8 XCDs round-robin, so with a multiple of 8 strips each
//     XCD takes every eighth strip across the grid's width, row chunk after
//     row chunk (the concurrent loads spread over the whole address range;
//     giving each XCD a contiguous run of strips instead kept the re-read
//     traffic unchanged and ran 1.4x slower);
//   * wrap-around indices are computed once per thread (columns) and once per
//     row (uniform), so the periodic boundary costs nothing per node.
#include "common.h"
#include "sem_internal.h"

namespace sem {

constexpr int FD_TX = 256;  // columns per workgroup (four waves)
constexpr int FD_P = 4;     // rows per pipeline step
constexpr int FD_RMAX = 7;
// rows per workgroup (a multiple of FD_P)
template <int R> constexpr int fd_rows() { return R <= 2 ? 16 : 32; }

struct FdArgs {
  const double *u_cur, *u_prev;
  double *u_next;
  int64_t nx, ny;
  uint32_t gx;  // strips (workgroups per row chunk)
  double c;
  double w[2 * FD_RMAX + 1];
};

// v mod n for v within a few periods of [0, n): on grids larger than the
// stencil one compare, no division (the row index is wrapped once per row)
__device__ inline int64_t fd_wrap(int64_t v, int64_t n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}

template <int R>
__global__ void __launch_bounds__(FD_TX) k_fd2d(FdArgs a) {
  // separate multiplies and adds in the stated order (no fused
  // multiply-add): at 24 bytes per node the kernel is bound by HBM, not by
  // the ~8r flops, and the update is then reproducible bit for bit
#pragma clang fp contract(off)
  constexpr int P = FD_P, Q = 2 * R + P, LW = FD_TX + 2 * R, ROWS = fd_rows<R>();
  __shared__ double rows[2][P][LW];
  const int tx = threadIdx.x;
  const int64_t nx = a.nx, ny = a.ny;
  // 32-bit decode of the block index (the grid has < 2^31 blocks)
  const uint32_t by = blockIdx.x / a.gx, bx = blockIdx.x - by * a.gx;
  const int64_t i0 = (int64_t)bx * FD_TX;
  const int64_t j0 = (int64_t)by * ROWS;
  const int64_t jend = j0 + ROWS < ny ? j0 + ROWS : ny;
  const bool act = i0 + tx < nx;
  // this thread's column and, for tx < R, one left and one right halo
  // column (all wrapped; lanes past nx carry wrapped values for the halo of
  // the last real column)
  auto wrap_col = [nx](int64_t v) {
    v %= nx;
    return v < 0 ? v + nx : v;
  };
  const int64_t ci = wrap_col(i0 + tx);
  const int64_t cl = tx < R ? wrap_col(i0 - R + tx) : 0;
  const int64_t cr = tx < R ? wrap_col(i0 + FD_TX + tx) : 0;
  const double *uc = a.u_cur;

  // q[m] holds u_cur(ci, j - R + m) for the current first row j
  double q[Q];
#pragma unroll
  for (int m = 0; m < 2 * R; ++m) q[m] = uc[fd_wrap(j0 - R + m, ny) * nx + ci];

  // loads of the rows j .. j + P - 1: the new window rows (j + R + p), the
  // previous level and, for tx < R, the halo columns of the centre rows
  double qn[P], upn[P], hl[P], hr[P];
  auto issue = [&](int64_t j) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      qn[p] = uc[fd_wrap(j + R + p, ny) * nx + ci];
      upn[p] = (act && j + p < jend)
                   ? __builtin_nontemporal_load(a.u_prev + (j + p) * nx + ci)
                   : 0.0;
      if (tx < R) {
        const int64_t jc = fd_wrap(j + p, ny) * nx;
        hl[p] = uc[jc + cl];
        hr[p] = uc[jc + cr];
      }
    }
  };
  issue(j0);
  int buf = 0;
  for (int64_t j = j0; j < jend; j += P) {  // uniform
    double up[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      q[2 * R + p] = qn[p];
      up[p] = upn[p];
      rows[buf][p][R + tx] = q[R + p];
      if (tx < R) {
        rows[buf][p][tx] = hl[p];
        rows[buf][p][R + FD_TX + tx] = hr[p];
      }
    }
    if (j + P < jend) issue(j + P);  // in flight during this step
    __syncthreads();
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double lap = 0.0;
#pragma unroll
      for (int k = -R; k <= R; ++k)
        lap += a.w[R + k] * rows[buf][p][R + tx + k] + a.w[R + k] * q[R + p + k];
      if (act && j + p < jend)
        __builtin_nontemporal_store(2.0 * q[R + p] - up[p] + a.c * lap,
                                    a.u_next + (j + p) * nx + ci);
    }
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) q[m] = q[m + P];
    buf ^= 1;
  }
}

// Unit-spacing weights of the second derivative, order 2r (closed forms of
// the maximal-order centred formula): w_k = 2 (-1)^(k+1) (r!)^2 /
// (k^2 (r-k)! (r+k)!) for k != 0 and w_0 = -2 sum_{k=1..r} 1/k^2.  For
// r <= 7 every numerator and denominator is an integer below 2^53, so each
// weight is one correctly rounded division of exact values.
void fd2d_weights_host(int r, double *w) {
  if (r < 1 || r > FD_RMAX) fail(SEM_ERR_ARG, "fd2d: r must be in 1..7");
  auto fact = [](int n) {
    int64_t f = 1;
    for (int m = 2; m <= n; ++m) f *= m;
    return f;
  };
  const int64_t rf = fact(r);
  int64_t lcm = 1;  // lcm(1..r)
  for (int k = 1; k <= r; ++k) {
    int64_t a = lcm, b = k;
    while (b) {
      const int64_t t = a % b;
      a = b;
      b = t;
    }
    lcm = lcm / a * k;
  }
  int64_t s = 0;  // sum_k (lcm / k)^2 = lcm^2 sum_k 1 / k^2
  for (int k = 1; k <= r; ++k) {
    const int64_t num = 2 * rf * rf, den = (int64_t)k * k * fact(r - k) * fact(r + k);
    const double v = (double)num / (double)den;
    w[r + k] = w[r - k] = (k % 2) ? v : -v;
    s += (lcm / k) * (lcm / k);
  }
  w[r] = -(double)(2 * s) / (double)(lcm * lcm);
}

void launch_fd2d(const double *u_cur, const double *u_prev, double *u_next,
                 int64_t nx, int64_t ny, int r, double c, hipStream_t s) {
  if (nx < 1 || ny < 1) fail(SEM_ERR_ARG, "fd2d: grid must have nx, ny >= 1");
  if (!u_cur || !u_prev || !u_next) fail(SEM_ERR_ARG, "fd2d: null buffer");
  if (u_next == u_cur) fail(SEM_ERR_ARG, "fd2d: u_next must not alias u_cur");
  const int rows = r <= 2 ? 16 : 32;  // fd_rows<r>()
  const int64_t gx = (nx + FD_TX - 1) / FD_TX, gy = (ny + rows - 1) / rows;
  if (gx * gy > INT32_MAX) fail(SEM_ERR_ARG, "fd2d: grid too large");
  FdArgs a{};
  a.u_cur = u_cur;
  a.u_prev = u_prev;
  a.u_next = u_next;
  a.nx = nx;
  a.ny = ny;
  a.gx = (uint32_t)gx;
  a.c = c;
  fd2d_weights_host(r, a.w);
  const dim3 grid((unsigned)(gx * gy)), block(FD_TX);
  switch (r) {
#define SEM_FD(RR)                                                    \
  case RR:                                                            \
    hipLaunchKernelGGL(k_fd2d<RR>, grid, block, 0, s, a);             \
    break;
    SEM_FD(1)
    SEM_FD(2)
    SEM_FD(3)
    SEM_FD(4)
    SEM_FD(5)
    SEM_FD(6)
    SEM_FD(7)
#undef SEM_FD
    default: fail(SEM_ERR_ARG, "fd2d: r must be in 1..7");
  }
  SEM_HIP(hipGetLastError());
}

}  // namespace sem
