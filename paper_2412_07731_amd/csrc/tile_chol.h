// Cholesky factor and its inverse for one 16x16 tile, computed by one wave.
//
// Gaussian elimination without pivoting on the augmented tile [P | I]: after
// the 16 steps the left half is U = D L_u' and the right half E = L_u^-1 for
// P = L_u D L_u'.  Scaling row j of both halves by 1/sqrt(d_j) gives L' and
// L^-1 of the Cholesky factor P = L L'.  A pivot d_j <= thr is replaced by a
// huge value (the pivot rule) and counted.
//
// Layout: lane l holds row i = l%16 and columns 4g..4g+3 (g = l/16) of both
// halves; row j and the multipliers of step j are exchanged through a small
// LDS buffer (48 values), so a step costs one division, a few LDS accesses and
// eight FMAs.  The caller's workgroup must be exactly this wave or the other
// waves must not touch xbuf.
#pragma once

#include "common.h"

namespace ahlp {

__device__ __forceinline__ void wave_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// workgroup barrier that orders LDS accesses only: the waves' global stores
// stay in flight across it
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ __forceinline__ T lane_bcast(T v, int src);
template <>
__device__ __forceinline__ double lane_bcast<double>(double v, int src) {
  union { double d; int i[2]; } u;
  u.d = v;
  u.i[0] = __builtin_amdgcn_readlane(u.i[0], src);
  u.i[1] = __builtin_amdgcn_readlane(u.i[1], src);
  return u.d;
}
template <>
__device__ __forceinline__ float lane_bcast<float>(float v, int src) {
  union { float f; int i; } u;
  u.f = v;
  u.i = __builtin_amdgcn_readlane(u.i, src);
  return u.f;
}

// P: input tile (column-major, LDS or global).  L (may alias P) receives the
// lower factor (upper part zero), Li its inverse; both column-major.  xbuf: 48
// values of LDS scratch.  Returns the number of replaced pivots (all lanes).
template <typename T>
__device__ __forceinline__ int wave_chol_tile(const T* P, T* L, T* Li, double thr, T* xbuf) {
  const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
  T a[4], e[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = P[(4 * g + r) * TS + i];
    e[r] = (4 * g + r == i) ? T(1) : T(0);
  }
  int cnt = 0;
  T mypiv = T(1);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    T p = lane_bcast<T>(a[j & 3], j + 16 * (j >> 2));
    if (!((double)p > thr)) {
      p = (T)PIVOT_BIG;
      ++cnt;
    }
    const T rp = T(1) / p;
    if (i == j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xbuf[4 * g + r] = a[r];
        xbuf[16 + 4 * g + r] = e[r];
      }
      mypiv = p;
    }
    if (g == (j >> 2)) xbuf[32 + i] = a[j & 3] * rp;
    wave_order();
    const T m = (i > j) ? xbuf[32 + i] : T(0);
    T rj[4], rje[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rj[r] = xbuf[4 * g + r];
      rje[r] = xbuf[16 + 4 * g + r];
    }
    wave_order();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] -= m * rj[r];
      e[r] -= m * rje[r];
    }
  }
  const T s = T(1) / (T)sqrt((double)mypiv);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = 4 * g + r;
    // L' row i = U row i * s, i.e. L[c][i] (zero above the diagonal); Li row i = E row i * s
    L[i * TS + c] = (c >= i) ? a[r] * s : T(0);
    Li[c * TS + i] = e[r] * s;
  }
  wave_order();
  return cnt;
}

}  // namespace ahlp
