// Border step of the Schur solve by cyclic reduction, shared by the one-tile
// and the two-tile pair kernels: after the forward reduction every pair j has
// left its border partial Z_j'w_j (16 t0 values) in pb.
#pragma once

#include "common.h"
#include "kernels.h"
#include "tile_ops.h"

namespace ahlp {

// s0 = s_0 - sum_j Z_j'w_j (chunks of pairs, then the chunks, in a fixed
// order), w0 = T Lb^-1 s0, u0 = -Lb^-T w0 (T = diag(-1 on the border's global
// rows, +1 on x_0), the signs of -(S00 - sum Z'Z) = Lb T Lb'); u0 goes to
// LDS, to A.u0p and to the border part of A.u.  Every thread of the workgroup calls it (it holds
// barriers); part: blockDim.x doubles, s0 / w0 / u0: 16 t0 each, sc: 16, all
// LDS.  Wave 0 does the triangular solves with the tiles of Lb^-1: lbi is
// either the factor's full t0 x t0 array (tile (r, c) at c t0 + r) or, if
// packed, a copy of its lower triangle (tile (r, c) at r (r + 1) / 2 + c).
__device__ __forceinline__ int lbi_tile(int r, int c, int t0, bool packed) {
  return packed ? r * (r + 1) / 2 + c : c * t0 + r;
}
__device__ inline void bcr_border_solve(const BcrSolveArgs& A, const double* lbi, bool packed,
                                        double* part, double* s0, double* w0, double* u0,
                                        double* sc) {
  const BcrArgs& c = A.c;
  const int t0 = c.t0, n0 = c.n0, nb = 16 * t0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (nb == 0) return;
  const int nch = blockDim.x / nb;
  const int ch = threadIdx.x / nb, i = threadIdx.x % nb;
  if (ch < nch) {
    const int per = (c.P + nch - 1) / nch;
    const int j0 = ch * per, j1 = min(c.P, j0 + per);
    double acc = 0.0;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) acc += A.pb[(long long)j * nb + i];
    part[ch * nb + i] = acc;
  }
  __syncthreads();
  if (threadIdx.x < nb) {
    double acc = 0.0;
    for (int ch2 = 0; ch2 < nch; ++ch2) acc += part[ch2 * nb + threadIdx.x];
    s0[threadIdx.x] = (threadIdx.x < n0 ? A.s[A.nl + threadIdx.x] : 0.0) - acc;
  }
  __syncthreads();
  if (wave == 0) {
    for (int rr = 0; rr < t0; ++rr) {
      double acc = 0.0;
      for (int cc = 0; cc <= rr; ++cc) acc += op_mv(op_load(lbi + lbi_tile(rr, cc, t0, packed) * 256), s0 + 16 * cc);
      wave_order();
      if (lane < 16) w0[16 * rr + lane] = (16 * rr + lane < c.ng) ? -acc : acc;
      wave_order();
    }
    for (int cc = 0; cc < t0; ++cc) {
      double acc = 0.0;
      for (int rr = cc; rr < t0; ++rr)
        acc += op_mtv(op_load(lbi + lbi_tile(rr, cc, t0, packed) * 256), w0 + 16 * rr, sc);
      if (lane < 16) {
        u0[16 * cc + lane] = -acc;
        A.u0p[16 * cc + lane] = -acc;
        if (16 * cc + lane < n0) A.u[A.nl + 16 * cc + lane] = -acc;
      }
      wave_order();
    }
  }
  __syncthreads();
}

}  // namespace ahlp
