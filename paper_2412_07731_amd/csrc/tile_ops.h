// One-wave operations on 16x16 FP64 tiles (column-major, 256 doubles) and on
// 16-vectors, built on the 16x16x4 FP64 MFMA.
//
// Operand layout of v_mfma_f64_16x16x4f64: for the s-th of four K-steps lane l
// supplies A(l%16, 4s + l/16) and B(4s + l/16, l%16); for a column-major tile X
// these are X[64 s + l] (A = X) and X[(l%16)*16 + 4s + l/16] (B = X).  The
// accumulator holds element (acc_row(l, r), l%16) in register r.
#pragma once

#include "common.h"
#include "tile_chol.h"

namespace ahlp {

struct Op { double v[4]; };   // a tile as an A operand: element 64 s + lane

__device__ __forceinline__ Op op_load(const double* t) {
  const int lane = threadIdx.x & 63;
  Op o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[64 * s + lane];
  return o;
}
__device__ __forceinline__ d4 acc_zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ d4 acc_load(const double* t) {
  const int lane = threadIdx.x & 63;
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = t[acc_index<double>(lane, r)];
  return a;
}
__device__ __forceinline__ void acc_store(double* t, d4 a) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[acc_index<double>(lane, r)] = a[r];
}
// padded tile of an exact column-major block (rows x cols, leading dimension
// ld); identity on the padded part of the diagonal if diag
__device__ __forceinline__ d4 acc_load_exact(const double* src, int rows, int cols, int ld,
                                             bool diag) {
  const int lane = threadIdx.x & 63;
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = acc_row<double>(lane, r), j = lane & 15;
    double v = 0.0;
    if (i < rows && j < cols) v = src[i + j * ld];
    else if (diag && i == j) v = 1.0;
    a[r] = v;
  }
  return a;
}
// transposed padded tile: element (i, j) = src[j + i*ld], i < rows, j < cols
__device__ __forceinline__ d4 acc_load_exact_t(const double* src, int rows, int cols, int ld) {
  const int lane = threadIdx.x & 63;
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = acc_row<double>(lane, r), j = lane & 15;
    a[r] = (i < rows && j < cols) ? src[j + i * ld] : 0.0;
  }
  return a;
}
// acc += alpha X Y'
__device__ __forceinline__ d4 mma_xyt(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(alpha * X[64 * s + lane], Y[64 * s + lane], acc);
  return acc;
}
// acc += alpha X S Y' with S = diag(-1 where neg has the bit of the inner
// index, +1 elsewhere)
__device__ __forceinline__ d4 mma_xsyt(d4 acc, const double* X, const double* Y, double alpha,
                                       unsigned neg) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double f = ((neg >> (4 * s + (lane >> 4))) & 1u) ? -alpha : alpha;
    acc = mfma(f * X[64 * s + lane], Y[64 * s + lane], acc);
  }
  return acc;
}
// acc += alpha X Y
__device__ __forceinline__ d4 mma_xy(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = mfma(alpha * X[64 * s + lane], Y[(lane & 15) * TS + 4 * s + (lane >> 4)], acc);
  return acc;
}
// acc += alpha X' Y
__device__ __forceinline__ d4 mma_txy(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
  const int idx = (lane & 15) * TS + (lane >> 4);
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(alpha * X[idx + 4 * s], Y[idx + 4 * s], acc);
  return acc;
}
__device__ __forceinline__ void tile_copy(double* dst, const double* src) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) dst[64 * s + lane] = src[64 * s + lane];
}

// y = X v (v: 16 values in LDS); every lane returns y[lane % 16]
__device__ __forceinline__ double op_mv(const Op& X, const double* v) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += X.v[k] * v[4 * k + (lane >> 4)];
  return col_sum4(s);
}
// y = X' v (v: 16 values in LDS); every lane returns y[lane % 16].  Row g of
// the wave sums column 4 s + g of X into out[s]; lane (i, any row) takes y[i]
// from row i % 4, whose lanes i & 12 .. (i & 12) + 3 hold out[i / 4] in the
// register the lane selects.  sc is not used (kept for the callers' layouts).
__device__ __forceinline__ double op_mtv(const Op& X, const double* v, double* sc) {
  (void)sc;
  const int lane = threadIdx.x & 63, i = lane & 15;
  const double vi = v[i];
  double out[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) out[s] = row_sum16(X.v[s] * vi);
  const int q = i >> 2;
  const double sel = q == 0 ? out[0] : q == 1 ? out[1] : q == 2 ? out[2] : out[3];
  return __shfl(sel, ((i & 3) << 4) | (i & 12));
}
__device__ __forceinline__ void vec_put(double* dst, double y) {
  const int lane = threadIdx.x & 63;
  if (lane < 16) dst[lane] = y;
}
// element lane % 16 of an exact vector of len values, zero past the end
__device__ __forceinline__ double vec_get_exact(const double* src, int len) {
  const int i = threadIdx.x & 15;
  return i < len ? src[i] : 0.0;
}

// Blocked Cholesky of a t x t matrix of tiles, by one wave.  B holds tile
// (r, c) at (c t + r) 256 (LDS; only tiles with r >= c are read).  On return
// those tiles hold the factor L, Ld the inverses of its t diagonal tiles and X
// (t x t tiles, zero above the diagonal) the block inverse L^-1.  tmp: one
// tile and xbuf 48 values of LDS scratch.  A pivot <= thr is replaced (the
// pivot rule); returns the number replaced (all lanes).  With neg != 0 (bit j:
// row j's sign is negative) B is quasi-definite and the factorization signed,
// B = L S L' with S = diag(-1 on neg's bits, +1 elsewhere): tile column p is
// L_rp = B_rp L_pp^-T S_p, and the trailing update subtracts L_rp S_p L_cp'.
__device__ inline int wave_block_chol(double* B, int t, double* X, double* Ld, double* tmp,
                                      double* xbuf, double thr, unsigned long long neg = 0) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int p = 0; p < t; ++p) {
    double* Bpp = B + (p * t + p) * 256;
    const unsigned np = (unsigned)((neg >> (16 * p)) & 0xFFFFull);
    if (neg) cnt += wave_chol_tile<double, TS, true>(Bpp, Bpp, Ld + p * 256, thr, xbuf, np);
    else cnt += wave_chol_tile<double>(Bpp, Bpp, Ld + p * 256, thr, xbuf);
    for (int r = p + 1; r < t; ++r) {
      d4 acc = mma_xyt(acc_zero(), B + (p * t + r) * 256, Ld + p * 256, 1.0);
      if (neg && ((np >> (lane & 15)) & 1u)) acc = -acc;   // times S_p (column lane % 16)
      wave_order();
      acc_store(B + (p * t + r) * 256, acc);
    }
    wave_order();
    for (int r = p + 1; r < t; ++r)
      for (int cc = p + 1; cc <= r; ++cc) {
        d4 acc = acc_load(B + (cc * t + r) * 256);
        if (neg) acc = mma_xsyt(acc, B + (p * t + r) * 256, B + (p * t + cc) * 256, -1.0, np);
        else acc = mma_xyt(acc, B + (p * t + r) * 256, B + (p * t + cc) * 256, -1.0);
        wave_order();
        acc_store(B + (cc * t + r) * 256, acc);
      }
    wave_order();
  }
  // X = L^-1 by block columns
  for (int cc = 0; cc < t; ++cc) {
    for (int r = 0; r < t; ++r) {
      if (r < cc) {
        for (int s = 0; s < 4; ++s) X[(cc * t + r) * 256 + 64 * s + lane] = 0.0;
      } else if (r == cc) {
        tile_copy(X + (cc * t + r) * 256, Ld + r * 256);
      } else {
        d4 acc = acc_zero();
        for (int q = cc; q < r; ++q) acc = mma_xy(acc, B + (q * t + r) * 256, X + (cc * t + q) * 256, 1.0);
        acc_store(tmp, acc);
        wave_order();
        d4 x = mma_xy(acc_zero(), Ld + r * 256, tmp, -1.0);
        wave_order();
        acc_store(X + (cc * t + r) * 256, x);
      }
      wave_order();
    }
  }
  return cnt;
}


}  // namespace ahlp
