// Index arithmetic of the structured box mesh, the closed form of the
// distinct global-local node numbering (paper section 4.2.1) for a
// lexicographic E_x x E_y x E_z box of order N:
//   element  e = ex + Ex (ey + Ey ez),
//   local    l = e n1^3 + i + n1 j + n1^2 k,          n1 = N + 1,
//   global   g = gx + Gx (gy + Gy gz),  gx = ex N + i (and y, z alike),
// with G_d = E_d N + 1 coordinates per direction, or G_d = E_d N in a
// periodic direction, whose faces at 0 and 1 are identified (the coordinate
// E_d N wraps to 0).
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
  int32_t N, n1, Ex, Ey, Ez, Gx, Gy, Gz, dirichlet, periodic;  // periodic: bit 1 x, 2 y, 4 z
  // order of the copy directions in ascending local index (copy_order);
  // mN = floor(2^32 / N) + 1 (0 for N = 1): the 32-bit quotient by N
  int32_t order;
  uint32_t mN;
  int64_t Gxy;
  FastDiv dEx, dEy, dGx, dGxy, dN;
};

// The copies of a global node are the combinations of at most two copies
// per direction.  In ascending local index l = e n1^3 + i + n1 j + n1^2 k
// they come direction by direction, the direction whose two copies differ
// most in l outermost: copies in different elements differ by at least
// one element (n1^3 > N (n1^2 + n1 + 1)), z more than y more than x; the
// two copies of a periodic direction with a single element lie in the
// same element (at node 0 and N) and differ by N, N n1 or N n1^2 only.
// Orders (outer to inner): 0 z y x, 1 y x z, 2 z x y, 3 x z y, 4 y z x.
inline int copy_order(int Ex, int Ey, int Ez, int periodic) {
  const bool wx = (periodic & 1) && Ex == 1, wy = (periodic & 2) && Ey == 1,
             wz = (periodic & 4) && Ez == 1;
  // element-level directions first (z, y, x), then the in-element ones
  // (z, y, x); an in-element x is innermost in either group
  if (wz && wy) return wx ? 0 : 3;  // x z y (all three in-element: z y x)
  if (wz) return wx ? 4 : 1;        // y z x, or y x z
  if (wy) return wx ? 0 : 2;        // z y x, or z x y
  return 0;
}

inline Box make_box(int N, int Ex, int Ey, int Ez, int dirichlet, int periodic) {
  Box b;
  b.N = N;
  b.n1 = N + 1;
  b.Ex = Ex;
  b.Ey = Ey;
  b.Ez = Ez;
  b.Gx = Ex * N + ((periodic & 1) ? 0 : 1);
  b.Gy = Ey * N + ((periodic & 2) ? 0 : 1);
  b.Gz = Ez * N + ((periodic & 4) ? 0 : 1);
  b.dirichlet = dirichlet;
  b.periodic = periodic;
  b.order = copy_order(Ex, Ey, Ez, periodic);
  b.mN = N <= 1 ? 0u : (uint32_t)((1ull << 32) / (uint64_t)N + 1);
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

// element coordinates (ex, ey, ez) of element e
struct ElemXYZ {
  uint32_t x, y, z;
};
__host__ __device__ inline ElemXYZ box_elem(const Box &b, uint32_t e) {
  const uint32_t t = fdiv(e, b.dEx), ex = e - t * (uint32_t)b.Ex;
  const uint32_t ez = fdiv(t, b.dEy), ey = t - ez * (uint32_t)b.Ey;
  return {ex, ey, ez};
}

// lattice coordinate c = e_d N + i (at most G_d) of one direction: in a
// periodic direction E_d N is coordinate 0; otherwise c < G_d already
__host__ __device__ inline uint32_t wrap_coord(uint32_t c, int32_t G) {
  return c == (uint32_t)G ? 0u : c;
}

// global index of node (i, j, k) of the element at coordinates c
__host__ __device__ inline int64_t box_node(const Box &b, const ElemXYZ &c, uint32_t i,
                                            uint32_t j, uint32_t k) {
  const uint32_t gx = wrap_coord(c.x * (uint32_t)b.N + i, b.Gx);
  const uint32_t gy = wrap_coord(c.y * (uint32_t)b.N + j, b.Gy);
  const uint32_t gz = wrap_coord(c.z * (uint32_t)b.N + k, b.Gz);
  return (int64_t)gx + (int64_t)b.Gx * ((int64_t)gy + (int64_t)b.Gy * gz);
}

// the copies of a node along one direction, in ascending element order:
// global coordinate x lies in element c0 at node index i0 and, when
// cnt == 2, also in element c1 at node index i1
struct AxisCopies {
  uint32_t c0, i0, c1, i1;
  int cnt;
};

__host__ __device__ inline AxisCopies axis_copies(uint32_t x, uint32_t E,
                                                  uint32_t N, const FastDiv &dN,
                                                  bool periodic) {
  // periodic: coordinate 0 is node 0 of element 0 and node N of element
  // E - 1 (the same element when E = 1: node 0 before node N)
  if (periodic && x == 0) return {0, 0, E - 1, N, 2};
  const uint32_t q = fdiv(x, dN), i = x - q * N;
  if (q == E) return {E - 1, N, 0, 0, 1};
  if (i == 0 && q > 0) return {q - 1, N, q, 0, 2};
  return {q, i, 0, 0, 1};
}

struct NodeCopies {
  AxisCopies x, y, z;
  bool masked;  // on the Dirichlet boundary
};

// PER = false: the caller knows that the box has no periodic direction
// (the compiler then drops the wrap-around cases)
template <bool PER = true>
__host__ __device__ inline NodeCopies node_copies(const Box &b, uint32_t g) {
  const uint32_t gz = fdiv(g, b.dGxy);
  const uint32_t rem = g - gz * (uint32_t)b.Gxy;
  const uint32_t gy = fdiv(rem, b.dGx), gx = rem - gy * (uint32_t)b.Gx;
  NodeCopies c;
  const bool px = PER && (b.periodic & 1), py = PER && (b.periodic & 2),
             pz = PER && (b.periodic & 4);
  c.x = axis_copies(gx, b.Ex, b.N, b.dN, px);
  c.y = axis_copies(gy, b.Ey, b.N, b.dN, py);
  c.z = axis_copies(gz, b.Ez, b.N, b.dN, pz);
  // Dirichlet faces: the outer faces of the non-periodic directions
  c.masked = b.dirichlet &&
             ((!px && (gx == 0 || gx == (uint32_t)b.Gx - 1)) ||
              (!py && (gy == 0 || gy == (uint32_t)b.Gy - 1)) ||
              (!pz && (gz == 0 || gz == (uint32_t)b.Gz - 1)));
  return c;
}

// local index of copy (a, bb, c) (each 0 or 1, below the counts)
__host__ __device__ inline int64_t copy_lid(const Box &b, const NodeCopies &nc,
                                            int a, int bb, int c) {
  const uint32_t ez = a ? nc.z.c1 : nc.z.c0, iz = a ? nc.z.i1 : nc.z.i0;
  const uint32_t ey = bb ? nc.y.c1 : nc.y.c0, iy = bb ? nc.y.i1 : nc.y.i0;
  const uint32_t ex = c ? nc.x.c1 : nc.x.c0, ix = c ? nc.x.i1 : nc.x.i0;
  const int64_t e = (int64_t)ex + (int64_t)b.Ex * ((int64_t)ey + (int64_t)b.Ey * ez);
  return e * b.n1 * b.n1 * b.n1 + ix + b.n1 * ((int64_t)iy + (int64_t)b.n1 * iz);
}

// ---------------------------------------------------------------------------
// The same enumeration in a form for the solver kernels, which visit many
// nodes per thread.  The local index l = e n1^3 + i + n1 j + n1^2 k with
// e = e_x + E_x (e_y + E_y e_z) is a sum of one term per direction,
// (e_x n1^3 + i) + (e_y E_x n1^3 + n1 j) + (e_z E_x E_y n1^3 + n1^2 k), so
// copy (a, b, c) of a node has l = Z[a] + Y[b] + X[c] from the (at most two)
// copy terms of each direction.  IT is the index type: 32-bit when every
// local index fits, else 64-bit.

// floor(x / N) by one 32-bit high multiply: with m = floor(2^32 / N) + 1 =
// (2^32 + d) / N, 0 < d <= N, the error x d / (N 2^32) stays below 1 / N for
// x < 2^32 / N, which the coordinates (at most E_d N + 1) satisfy
__host__ __device__ inline uint32_t div_order(const Box &b, uint32_t x) {
  if (b.mN == 0) return x;
#ifdef __HIP_DEVICE_COMPILE__
  return __umulhi(x, b.mN);
#else
  return (uint32_t)(((uint64_t)x * b.mN) >> 32);
#endif
}

template <class IT> struct AxisTerms {
  IT t0, t1;  // local-index terms of the first and (cnt == 2) second copy
  int cnt;
};

// the cases of axis_copies, as index terms: se = the element stride of the
// direction in l, sn = its node stride
template <class IT>
__host__ __device__ inline AxisTerms<IT> axis_terms(const Box &b, uint32_t x, uint32_t E,
                                                    bool periodic, IT se, IT sn) {
  const uint32_t N = (uint32_t)b.N, q = div_order(b, x), i = x - q * N;
  uint32_t c0 = q, i0 = i, c1 = 0, i1 = 0;
  int cnt = 1;
  if (periodic && x == 0) {
    c0 = 0, i0 = 0, c1 = E - 1, i1 = N, cnt = 2;
  } else if (q == E) {
    c0 = E - 1, i0 = N;
  } else if (i == 0 && q > 0) {
    c0 = q - 1, i0 = N, c1 = q, cnt = 2;
  }
  return {(IT)c0 * se + (IT)i0 * sn, (IT)c1 * se + (IT)i1 * sn, cnt};
}

struct Coord3 {
  uint32_t x, y, z;
};

// global coordinates of node g
__host__ __device__ inline Coord3 box_coord(const Box &b, uint32_t g) {
  const uint32_t gz = fdiv(g, b.dGxy);
  const uint32_t rem = g - gz * (uint32_t)b.Gxy;
  const uint32_t gy = fdiv(rem, b.dGx);
  return {rem - gy * (uint32_t)b.Gx, gy, gz};
}

// advance coordinates by a fixed node step s, given as box_coord(s) (s =
// z Gxy + y Gx + x with x < G_x, y < G_y): one carry per direction
__host__ __device__ inline void box_advance(const Box &b, const Coord3 &s, Coord3 &p) {
  p.x += s.x;
  const uint32_t cx = p.x >= (uint32_t)b.Gx ? 1u : 0u;
  p.x -= cx * (uint32_t)b.Gx;
  p.y += s.y + cx;
  const uint32_t cy = p.y >= (uint32_t)b.Gy ? 1u : 0u;
  p.y -= cy * (uint32_t)b.Gy;
  p.z += s.z + cy;
}

template <class IT> struct CopyTerms {
  AxisTerms<IT> x, y, z;
  bool masked;  // on the Dirichlet boundary
};

template <class IT, bool PER>
__host__ __device__ inline CopyTerms<IT> copy_terms(const Box &b, const Coord3 &p) {
  const bool px = PER && (b.periodic & 1), py = PER && (b.periodic & 2),
             pz = PER && (b.periodic & 4);
  const IT n1 = (IT)b.n1, n3 = n1 * n1 * n1;
  CopyTerms<IT> c;
  c.x = axis_terms<IT>(b, p.x, (uint32_t)b.Ex, px, n3, (IT)1);
  c.y = axis_terms<IT>(b, p.y, (uint32_t)b.Ey, py, n3 * (IT)b.Ex, n1);
  c.z = axis_terms<IT>(b, p.z, (uint32_t)b.Ez, pz, n3 * (IT)b.Ex * (IT)b.Ey, n1 * n1);
  c.masked = b.dirichlet &&
             ((!px && (p.x == 0 || p.x == (uint32_t)b.Gx - 1)) ||
              (!py && (p.y == 0 || p.y == (uint32_t)b.Gy - 1)) ||
              (!pz && (p.z == 0 || p.z == (uint32_t)b.Gz - 1)));
  return c;
}

// sum of the (up to 8) copies of a node, v[4 a + 2 b + c] holding copy a
// along z, b along y, c along x (+0.0 for an absent copy, which leaves the
// sum unchanged bit for bit: it starts at +0.0 and so is never -0.0), in
// ascending local index: the box's direction order (copy_order)
template <class TV> __host__ __device__ inline TV sum_copies(int order, const TV (&v)[8]) {
  TV s = TV(0);
#define SEM_SUM3(A, B, C)                                  \
  _Pragma("unroll") for (int A = 0; A < 2; ++A)            \
    _Pragma("unroll") for (int B = 0; B < 2; ++B)          \
      _Pragma("unroll") for (int C = 0; C < 2; ++C) s = s + v[4 * a + 2 * b + c];
  switch (order) {
    case 0: {
      SEM_SUM3(a, b, c)
      break;
    }
    case 1: {
      SEM_SUM3(b, c, a)
      break;
    }
    case 2: {
      SEM_SUM3(a, c, b)
      break;
    }
    case 3: {
      SEM_SUM3(c, a, b)
      break;
    }
    default: {
      SEM_SUM3(b, a, c)
      break;
    }
  }
#undef SEM_SUM3
  return s;
}

}  // namespace sem
