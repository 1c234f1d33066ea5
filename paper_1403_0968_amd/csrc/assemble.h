// The assembled value w_G = mask o Q^T w_L at one global node (paper section
// 4.2.1, distinct global-local numbering): the node's copies in the E-vector
// w_L, found in closed form from its box coordinates (structured.h), summed
// from +0.0 in ascending local index; zero on Dirichlet nodes.
#pragma once

#include "common.h"
#include "structured.h"

namespace sem {

// all (up to 8) copies are loaded at once, predicated on existence (with the
// normal cache hint: a line of w_L holds copies of two rows of global nodes,
// which different threads assemble; non-temporal loads made the FP32
// assembly 52 -> 76 us); an
// absent copy adds +0.0, which leaves the sum unchanged bit for bit (the
// sum starts at +0.0 and so is never -0.0).  IT: the local index type
// (32-bit when every local index fits)
template <class TV, bool PER, class IT>
__device__ __forceinline__ TV assemble_node(const Box &bx, gp<const TV> wL, const Coord3 &pc) {
  const CopyTerms<IT> ct = copy_terms<IT, PER>(bx, pc);
  TV sw = TV(0);
  if (!ct.masked) {
    TV v[8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const bool ok = a < ct.z.cnt && b < ct.y.cnt && c < ct.x.cnt;
          const IT lid = (a ? ct.z.t1 : ct.z.t0) + (b ? ct.y.t1 : ct.y.t0) +
                         (c ? ct.x.t1 : ct.x.t0);
          v[4 * a + 2 * b + c] = ok ? wL[lid] : TV(0);
        }
    sw = sum_copies(PER ? bx.order : 0, v);
  }
  return sw;
}

}  // namespace sem
