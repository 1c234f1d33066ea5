// Index arithmetic of the structured box mesh, the closed form of the
// distinct global-local node numbering (paper section 4.2.1) for a
// lexicographic E_x x E_y x E_z box of order N:
//   element  e = ex + Ex (ey + Ey ez),
//   local    l = e n1^3 + i + n1 j + n1^2 k,          n1 = N + 1,
//   global   g = (ex N + i) + Gx ((ey N + j) + Gy (ez N + k)),  G_d = E_d N + 1.
// The solvers use it in place of the l2g / perm / offsets arrays (the
// arrays stay the reference numbering of sem_gs and the exports): a global
// node's local copies are enumerated in ascending local index, the order
// the array-based summation uses, so both give the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sem {

// unsigned 32-bit division by an invariant divisor through one 64 x 64 -> 128
// high multiply (Granlund and Montgomery 1994): with m = floor((2^64-1)/d)+1,
// floor(n m / 2^64) = floor(n / d) for all n, d < 2^32
struct FastDiv {
  uint64_t m;  // 0 encodes d == 1
  uint32_t d, pad;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.pad = 0;
  f.m = d <= 1 ? 0 : UINT64_MAX / d + 1;
  return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f) {
  if (f.m == 0) return n;
#ifdef __HIP_DEVICE_COMPILE__
  return (uint32_t)__umul64hi((uint64_t)n, f.m);
#else
  return (uint32_t)(((unsigned __int128)n * f.m) >> 64);
#endif
}

struct Box {
  int32_t N, n1, Ex, Ey, Ez, Gx, Gy, Gz, dirichlet, pad;
  int64_t Gxy;
  FastDiv dEx, dEy, dGx, dGxy, dN;
};

inline Box make_box(int N, int Ex, int Ey, int Ez, int dirichlet) {
  Box b;
  b.N = N;
  b.n1 = N + 1;
  b.Ex = Ex;
  b.Ey = Ey;
  b.Ez = Ez;
  b.Gx = Ex * N + 1;
  b.Gy = Ey * N + 1;
  b.Gz = Ez * N + 1;
  b.dirichlet = dirichlet;
  b.pad = 0;
  b.Gxy = (int64_t)b.Gx * b.Gy;
  b.dEx = make_fastdiv((uint32_t)Ex);
  b.dEy = make_fastdiv((uint32_t)Ey);
  b.dGx = make_fastdiv((uint32_t)b.Gx);
  b.dGxy = make_fastdiv((uint32_t)b.Gxy);
  b.dN = make_fastdiv((uint32_t)N);
  return b;
}

// global index of the node (0, 0, 0) of element e
__host__ __device__ inline int64_t box_origin(const Box &b, uint32_t e) {
  const uint32_t t = fdiv(e, b.dEx), ex = e - t * (uint32_t)b.Ex;
  const uint32_t ez = fdiv(t, b.dEy), ey = t - ez * (uint32_t)b.Ey;
  return (int64_t)ex * b.N +
         (int64_t)b.Gx * ((int64_t)ey * b.N + (int64_t)b.Gy * ((int64_t)ez * b.N));
}

// the copies of a node along one direction: global coordinate x in [0, E N]
// lies in element c0 at node index i0 and, when cnt == 2, also in element
// c0 + 1 at node index 0 (ascending element order)
struct AxisCopies {
  uint32_t c0, i0;
  int cnt;
};

__host__ __device__ inline AxisCopies axis_copies(uint32_t x, uint32_t E,
                                                  uint32_t N, const FastDiv &dN) {
  const uint32_t q = fdiv(x, dN), i = x - q * N;
  if (q == E) return {E - 1, N, 1};
  if (i == 0 && q > 0) return {q - 1, N, 2};
  return {q, i, 1};
}

struct NodeCopies {
  AxisCopies x, y, z;
  bool masked;  // on the Dirichlet boundary
};

__host__ __device__ inline NodeCopies node_copies(const Box &b, uint32_t g) {
  const uint32_t gz = fdiv(g, b.dGxy);
  const uint32_t rem = g - gz * (uint32_t)b.Gxy;
  const uint32_t gy = fdiv(rem, b.dGx), gx = rem - gy * (uint32_t)b.Gx;
  NodeCopies c;
  c.x = axis_copies(gx, b.Ex, b.N, b.dN);
  c.y = axis_copies(gy, b.Ey, b.N, b.dN);
  c.z = axis_copies(gz, b.Ez, b.N, b.dN);
  c.masked = b.dirichlet &&
             (gx == 0 || gy == 0 || gz == 0 || gx == (uint32_t)b.Gx - 1 ||
              gy == (uint32_t)b.Gy - 1 || gz == (uint32_t)b.Gz - 1);
  return c;
}

// local index of copy (a, bb, c) (each 0 or 1, below the counts)
__host__ __device__ inline int64_t copy_lid(const Box &b, const NodeCopies &nc,
                                            int a, int bb, int c) {
  const uint32_t ez = nc.z.c0 + a, iz = a ? 0 : nc.z.i0;
  const uint32_t ey = nc.y.c0 + bb, iy = bb ? 0 : nc.y.i0;
  const uint32_t ex = nc.x.c0 + c, ix = c ? 0 : nc.x.i0;
  const int64_t e = (int64_t)ex + (int64_t)b.Ex * ((int64_t)ey + (int64_t)b.Ey * ez);
  return e * b.n1 * b.n1 * b.n1 + ix + b.n1 * ((int64_t)iy + (int64_t)b.n1 * iz);
}

}  // namespace sem
