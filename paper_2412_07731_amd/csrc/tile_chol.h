// Cholesky factor and its inverse for one 16x16 tile, computed by one wave.
//
// Gaussian elimination without pivoting on the augmented tile [P | I]: after
// the 16 steps the left half is U = D L_u' and the right half E = L_u^-1 for
// P = L_u D L_u'.  Scaling row j of both halves by 1/sqrt(d_j) gives L' and
// L^-1 of the Cholesky factor P = L L'.  A pivot d_j <= thr is replaced by a
// huge value (the pivot rule) and counted.
//
// Both halves share one 16x16 array C: U is upper triangular and E unit lower
// triangular, and step j zeroes column j of U below the diagonal exactly where
// E gets its first nonzero there.  So C holds U on and above the diagonal and
// E below it; at step j row i > j is updated with the pivot row of C (its
// part left of column j is row j of E, its part right of it row j of U) and
// its entry in column j becomes E's, -m_ij.  Every value is the one the
// separate halves produce, with half the broadcasts and FMAs per step.
//
// Layout: lane l holds row i = l%16 and columns 4g..4g+3 (g = l/16).  At step
// j the 16-lane row g already holds columns 4g..4g+3 of every tile row, so row
// j reaches its lanes by a DPP row broadcast (row_newbcast:j) and the
// multiplier a_ij / d_j of row i comes from lane (i, j/4) by two cross-row
// swaps (permlane16, then permlane32): a step costs one reciprocal, the swaps,
// eight DPP moves and four FMAs, with no LDS round trip.
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

// value of lane J of each 16-lane row, in every lane of that row
// (row_newbcast writes every lane, so the move needs no old value; it is the
// one DPP control with a 64-bit move, one instruction for a double)
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
  const long long x = __builtin_bit_cast(long long, v);
  const long long y = __builtin_amdgcn_mov_dpp(x, 0x150 + J, 0xF, 0xF, false);
  return __builtin_bit_cast(double, y);
}
template <int J>
__device__ __forceinline__ float row_bcast(float v) {
  union { float f; int i; } u, o;
  u.f = v;
  o.i = __builtin_amdgcn_mov_dpp(u.i, 0x150 + J, 0xF, 0xF, false);
  return o.f;
}

// Value of row group K (lanes 16K..16K+15) in every row group, lane for lane:
// lane l receives v of lane 16K + l%16.  Two swap steps on the VALU (the
// permlane16 swap pairs rows 0/1 and 2/3, the permlane32 swap the half
// waves), instead of a permute through the LDS pipe.
template <int K>
__device__ __forceinline__ unsigned rowgroup_bcast_u32(unsigned v) {
  const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  const unsigned y = (K & 1) ? a[1] : a[0];   // [r0 r0 r2 r2] or [r1 r1 r3 r3]
  const auto b = __builtin_amdgcn_permlane32_swap(y, y, false, false);
  return (K & 2) ? b[1] : b[0];
}
template <int K>
__device__ __forceinline__ double rowgroup_bcast(double v) {
  union { double d; unsigned i[2]; } u;
  u.d = v;
  u.i[0] = rowgroup_bcast_u32<K>(u.i[0]);
  u.i[1] = rowgroup_bcast_u32<K>(u.i[1]);
  return u.d;
}
template <int K>
__device__ __forceinline__ float rowgroup_bcast(float v) {
  union { float f; unsigned i; } u;
  u.f = v;
  u.i = rowgroup_bcast_u32<K>(u.i);
  return u.f;
}

// 1 / p.  FP64: the hardware reciprocal estimate refined by two
// Newton-Raphson steps (r <- r + r (1 - p r), each doubling the correct
// bits), a few dependent instructions against the longer correctly rounded
// division sequence on the step's critical path (pivots are finite: a
// replaced one is 1e128).  FP32 keeps the division, since a replaced pivot is
// infinite there and 1 / inf must be 0.
__device__ __forceinline__ double recip(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  return fma(r, fma(-p, r, 1.0), r);
}
__device__ __forceinline__ float recip(float p) { return 1.0f / p; }

// Elimination step J on the lane's row i, column group g, of the combined
// array a.  SG: signed (quasi-definite) form, where column J's pivot must have
// the sign of its bit in neg (set: negative); the rule applies to the pivot
// times that sign.
template <typename T, int J, bool SG>
__device__ __forceinline__ void chol_step(T (&a)[4], int i, int g, double thr, int& cnt,
                                          T& mypiv, unsigned neg) {
  T p = lane_bcast<T>(a[J & 3], J + 16 * (J >> 2));
  if constexpr (SG) {
    const T tj = ((neg >> J) & 1u) ? T(-1) : T(1);
    if (!((double)(tj * p) > thr)) {
      p = tj * (T)PIVOT_BIG;
      ++cnt;
    }
  } else {
    if (!((double)p > thr)) {
      p = (T)PIVOT_BIG;
      ++cnt;
    }
  }
  const T rp = recip(p);
  if (i == J) mypiv = p;
  // a_iJ from lane (i, J/4); row J from lane J of this lane's 16-lane row
  const T aij = rowgroup_bcast<J / 4>(a[J & 3]);
  T rj[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) rj[r] = row_bcast<J>(a[r]);
  const T m = (i > J) ? aij * rp : T(0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T u = a[r] - m * rj[r];
    // column J of a row below the pivot: E's entry 0 - m * E(J, J) = 0 - m
    a[r] = (r == (J & 3) && g == (J >> 2) && i > J) ? T(0) - m : u;
  }
}
template <typename T, int J, bool SG>
__device__ __forceinline__ void chol_steps(T (&a)[4], int i, int g, double thr, int& cnt,
                                           T& mypiv, unsigned neg) {
  if constexpr (J < 16) {
    chol_step<T, J, SG>(a, i, g, thr, cnt, mypiv, neg);
    chol_steps<T, J + 1, SG>(a, i, g, thr, cnt, mypiv, neg);
  }
}

// P: input tile (column-major with leading dimension LD, LDS or global).  L
// (may alias P) receives the lower factor (upper part zero), Li its inverse;
// both column-major with leading dimension LD.  xbuf is no longer used (kept
// in the signature for the callers' LDS layouts).  Returns the number of
// replaced pivots (all lanes).  SG: the signed factorization of a
// quasi-definite tile, P = L S L' with S = diag(-1 where neg has the column's
// bit, +1 elsewhere); with D the elimination's pivots, L = L1 |D|^(1/2).
template <typename T, int LD = TS, bool SG = false>
__device__ __forceinline__ int wave_chol_tile(const T* P, T* L, T* Li, double thr, T* xbuf,
                                              unsigned neg = 0) {
  (void)xbuf;
  const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
  T a[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = P[(4 * g + r) * LD + i];
  int cnt = 0;
  T mypiv = T(1);
  chol_steps<T, 0, SG>(a, i, g, thr, cnt, mypiv, neg);
  T si = T(1);
  if constexpr (SG) {
    si = ((neg >> i) & 1u) ? T(-1) : T(1);
    mypiv *= si;
  }
  const T s = T(1) / (T)sqrt((double)mypiv);
  const T sl = SG ? si * s : s;
  wave_order();   // every lane has read P before L (which may alias it) is written
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = 4 * g + r;
    // L' row i = U row i * s (times the row's sign if SG), i.e. L[c][i] (zero
    // above the diagonal); Li row i = E row i * s (E: unit diagonal, zero
    // above it)
    const T e = c < i ? a[r] : (c == i ? T(1) : T(0));
    L[i * LD + c] = (c >= i) ? a[r] * sl : T(0);
    Li[c * LD + i] = e * s;
  }
  wave_order();
  return cnt;
}

}  // namespace ahlp
