// Host build of the closed-form box numbering that the solver kernels use
// (paper section 4.2.1, distinct global-local numbering), for the CPU tests:
// the maps it implies, and a self-check of the per-direction index terms,
// the carry stepping of coordinates and the 32-bit quotient by N against
// the plain enumeration of the same header.
#include "../../paper_1403_0968_amd/csrc/structured.h"

using namespace sem;

namespace {
// the summation order of the solver kernels: directions (a = z, b = y,
// c = x) nested outer to inner as copy_order lists them
const int kOrder[5][3] = {{0, 1, 2}, {1, 2, 0}, {0, 2, 1}, {2, 0, 1}, {1, 0, 2}};

template <bool PER>
long check_box(int N, int Ex, int Ey, int Ez, int dir, int per, uint32_t step) {
  const Box b = make_box(N, Ex, Ey, Ez, dir, per);
  const uint32_t nG = (uint32_t)((int64_t)b.Gx * b.Gy * b.Gz);
  long bad = 0;
  for (uint32_t g = 0; g < nG; ++g) {
    const NodeCopies nc = node_copies<PER>(b, g);
    const CopyTerms<uint32_t> t32 = copy_terms<uint32_t, PER>(b, box_coord(b, g));
    const CopyTerms<int64_t> t64 = copy_terms<int64_t, PER>(b, box_coord(b, g));
    if (nc.masked != t32.masked || nc.x.cnt != t32.x.cnt || nc.y.cnt != t32.y.cnt ||
        nc.z.cnt != t32.z.cnt || t64.x.cnt != t32.x.cnt) {
      ++bad;
      continue;
    }
    for (int a = 0; a < nc.z.cnt; ++a)
      for (int bb = 0; bb < nc.y.cnt; ++bb)
        for (int c = 0; c < nc.x.cnt; ++c) {
          const int64_t ref = copy_lid(b, nc, a, bb, c);
          const uint32_t l32 = (a ? t32.z.t1 : t32.z.t0) + (bb ? t32.y.t1 : t32.y.t0) +
                               (c ? t32.x.t1 : t32.x.t0);
          const int64_t l64 = (a ? t64.z.t1 : t64.z.t0) + (bb ? t64.y.t1 : t64.y.t0) +
                              (c ? t64.x.t1 : t64.x.t0);
          if ((int64_t)l32 != ref || l64 != ref) ++bad;
        }
  }
  const Coord3 s = box_coord(b, step);
  for (uint32_t g0 = 0; g0 < nG && g0 < 97; g0 += 7) {
    Coord3 p = box_coord(b, g0);
    for (uint32_t g = g0; g < nG; g += step) {
      const Coord3 q = box_coord(b, g);
      if (p.x != q.x || p.y != q.y || p.z != q.z) {
        ++bad;
        break;
      }
      box_advance(b, s, p);
    }
  }
  return bad;
}
}  // namespace

extern "C" {

// mismatches of the kernels' index arithmetic against the plain enumeration
// over boxes of every order 1..8, E_d in 1..3, both boundary kinds and all
// periodic combinations, node steps 1, 5, 64 and 256; and of the quotient
// by N on [0, 2^20) and just below 2^29
long structured_self_check() {
  long bad = 0;
  const uint32_t steps[4] = {1, 5, 64, 256};
  int k = 0;
  for (int N = 1; N <= 8; ++N)
    for (int Ex = 1; Ex <= 3; ++Ex)
      for (int Ey = 1; Ey <= 3; ++Ey)
        for (int Ez = 1; Ez <= 2; ++Ez)
          for (int dir = 0; dir <= 1; ++dir)
            for (int per = 0; per < 8; ++per) {
              const uint32_t st = steps[k++ % 4];
              bad += check_box<true>(N, Ex, Ey, Ez, dir, per, st);
              if (per == 0) bad += check_box<false>(N, Ex, Ey, Ez, dir, per, st);
            }
  for (int N = 1; N <= 8; ++N) {
    const Box b = make_box(N, 1, 1, 1, 1, 0);
    for (uint32_t x = 0; x < (1u << 20); ++x) bad += div_order(b, x) != x / (uint32_t)N;
    for (uint32_t x = (1u << 29) - 65536; x < (1u << 29); ++x)
      bad += div_order(b, x) != x / (uint32_t)N;
  }
  return bad;
}

// the sorted map (perm, offsets) and the Dirichlet flags of every global
// node as the solver kernels enumerate them: copies in summation order,
// local indices from the per-direction terms, coordinates stepped by one
// node with carries
void structured_maps(int N, int Ex, int Ey, int Ez, int dir, int per, int32_t *perm,
                     int32_t *offsets, uint8_t *gmask) {
  const Box b = make_box(N, Ex, Ey, Ez, dir, per);
  const uint32_t nG = (uint32_t)((int64_t)b.Gx * b.Gy * b.Gz);
  const Coord3 one = box_coord(b, 1);
  Coord3 p = box_coord(b, 0);
  int32_t pos = 0;
  for (uint32_t g = 0; g < nG; ++g, box_advance(b, one, p)) {
    const CopyTerms<int64_t> t = copy_terms<int64_t, true>(b, p);
    offsets[g] = pos;
    gmask[g] = t.masked;
    const int cnt[3] = {t.z.cnt, t.y.cnt, t.x.cnt};
    const int *o = kOrder[b.order];
    int q[3];
    for (q[0] = 0; q[0] < 2; ++q[0])
      for (q[1] = 0; q[1] < 2; ++q[1])
        for (q[2] = 0; q[2] < 2; ++q[2]) {
          int abc[3];
          abc[o[0]] = q[0];
          abc[o[1]] = q[1];
          abc[o[2]] = q[2];
          if (abc[0] < cnt[0] && abc[1] < cnt[1] && abc[2] < cnt[2])
            perm[pos++] = (int32_t)((abc[0] ? t.z.t1 : t.z.t0) + (abc[1] ? t.y.t1 : t.y.t0) +
                                    (abc[2] ? t.x.t1 : t.x.t0));
        }
  }
  offsets[nG] = pos;
}
}
