// One-wave operations on 16x16 FP64 tiles (column-major, 256 doubles) and on
// 16-vectors, built on the 16x16x4 FP64 MFMA.
//
// Operand layout of v_mfma_f64_16x16x4f64: for the s-th of four K-steps lane l
// supplies A(l%16, 4s + l/16) and B(4s + l/16, l%16); for a column-major tile X
// these are X[64 s + l] (A = X) and X[(l%16)*16 + 4s + l/16] (B = X).  The
// accumulator holds element (acc_row(l, r), l%16) in register r.
//
// The tile helpers take the leading dimension LD as a template argument
// (default 16, a dense 256-value tile).  LDS tiles with LD = 17 pad each
// column by one value: the accumulator-layout and B-operand accesses then
// spread the 16 lanes of a row group over distinct banks, where LD = 16 puts
// them all in one.  A padded tile takes 16 * 17 values.
#pragma once

#include "common.h"
#include "tile_chol.h"

namespace ahlp {

struct Op { double v[4]; };   // a tile as an A operand: element 64 s + lane

// offset of element (i, j) of a tile with leading dimension LD
template <int LD = TS>
__device__ __forceinline__ int tix(int i, int j) { return j * LD + i; }

template <int LD = TS>
__device__ __forceinline__ Op op_load(const double* t) {
  const int lane = threadIdx.x & 63;
  Op o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[tix<LD>(lane & 15, 4 * s + (lane >> 4))];
  return o;
}
template <int LD = TS>
__device__ __forceinline__ void op_store(double* t, const Op& o) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) t[tix<LD>(lane & 15, 4 * s + (lane >> 4))] = o.v[s];
}
__device__ __forceinline__ d4 acc_zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
template <int LD = TS>
__device__ __forceinline__ d4 acc_load(const double* t) {
  const int lane = threadIdx.x & 63;
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = t[tix<LD>(acc_row<double>(lane, r), lane & 15)];
  return a;
}
template <int LD = TS>
__device__ __forceinline__ void acc_store(double* t, d4 a) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[tix<LD>(acc_row<double>(lane, r), lane & 15)] = a[r];
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
template <int LD = TS>
__device__ __forceinline__ d4 mma_xyt(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int o = tix<LD>(lane & 15, 4 * s + (lane >> 4));
    acc = mfma(alpha * X[o], Y[o], acc);
  }
  return acc;
}
// acc += alpha X S Y' with S = diag(-1 where neg has the bit of the inner
// index, +1 elsewhere)
template <int LD = TS>
__device__ __forceinline__ d4 mma_xsyt(d4 acc, const double* X, const double* Y, double alpha,
                                       unsigned neg) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double f = ((neg >> (4 * s + (lane >> 4))) & 1u) ? -alpha : alpha;
    const int o = tix<LD>(lane & 15, 4 * s + (lane >> 4));
    acc = mfma(f * X[o], Y[o], acc);
  }
  return acc;
}
// acc += alpha X Y
template <int LD = TS>
__device__ __forceinline__ d4 mma_xy(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = mfma(alpha * X[tix<LD>(lane & 15, 4 * s + (lane >> 4))],
               Y[tix<LD>(4 * s + (lane >> 4), lane & 15)], acc);
  return acc;
}
// acc += alpha X' Y
template <int LD = TS>
__device__ __forceinline__ d4 mma_txy(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int o = tix<LD>(4 * s + (lane >> 4), lane & 15);
    acc = mfma(alpha * X[o], Y[o], acc);
  }
  return acc;
}
// tile copy between leading dimensions LDD (destination) and LDS_ (source)
template <int LDD = TS, int LDS_ = TS>
__device__ __forceinline__ void tile_copy(double* dst, const double* src) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = lane & 15, j = 4 * s + (lane >> 4);
    dst[tix<LDD>(i, j)] = src[tix<LDS_>(i, j)];
  }
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
// (r, c) at (c t + r) 16 LD (LDS; only tiles with r >= c are read).  On return
// those tiles hold the factor L, Ld the inverses of its t diagonal tiles and X
// (t x t tiles, zero above the diagonal) the block inverse L^-1.  tmp: one
// tile of LDS scratch (xbuf is not used); every tile has leading dimension LD.
// A pivot <= thr is replaced (the pivot rule); returns the number replaced
// (all lanes).  With neg != 0 (bit j:
// row j's sign is negative) B is quasi-definite and the factorization signed,
// B = L S L' with S = diag(-1 on neg's bits, +1 elsewhere): tile column p is
// L_rp = B_rp L_pp^-T S_p, and the trailing update subtracts L_rp S_p L_cp'.
template <int LD = TS>
__device__ inline int wave_block_chol(double* B, int t, double* X, double* Ld, double* tmp,
                                      double* xbuf, double thr, unsigned long long neg = 0) {
  constexpr int TT = 16 * LD;   // values per tile
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int p = 0; p < t; ++p) {
    double* Bpp = B + (p * t + p) * TT;
    const unsigned np = (unsigned)((neg >> (16 * p)) & 0xFFFFull);
    if (neg) cnt += wave_chol_tile<double, LD, true>(Bpp, Bpp, Ld + p * TT, thr, xbuf, np);
    else cnt += wave_chol_tile<double, LD>(Bpp, Bpp, Ld + p * TT, thr, xbuf);
    for (int r = p + 1; r < t; ++r) {
      d4 acc = mma_xyt<LD>(acc_zero(), B + (p * t + r) * TT, Ld + p * TT, 1.0);
      if (neg && ((np >> (lane & 15)) & 1u)) acc = -acc;   // times S_p (column lane % 16)
      wave_order();
      acc_store<LD>(B + (p * t + r) * TT, acc);
    }
    wave_order();
    for (int r = p + 1; r < t; ++r)
      for (int cc = p + 1; cc <= r; ++cc) {
        d4 acc = acc_load<LD>(B + (cc * t + r) * TT);
        if (neg) acc = mma_xsyt<LD>(acc, B + (p * t + r) * TT, B + (p * t + cc) * TT, -1.0, np);
        else acc = mma_xyt<LD>(acc, B + (p * t + r) * TT, B + (p * t + cc) * TT, -1.0);
        wave_order();
        acc_store<LD>(B + (cc * t + r) * TT, acc);
      }
    wave_order();
  }
  // X = L^-1 by block columns
  for (int cc = 0; cc < t; ++cc) {
    for (int r = 0; r < t; ++r) {
      if (r < cc) {
        op_store<LD>(X + (cc * t + r) * TT, Op{});
      } else if (r == cc) {
        tile_copy<LD, LD>(X + (cc * t + r) * TT, Ld + r * TT);
      } else {
        d4 acc = acc_zero();
        for (int q = cc; q < r; ++q) acc = mma_xy<LD>(acc, B + (q * t + r) * TT, X + (cc * t + q) * TT, 1.0);
        acc_store<LD>(tmp, acc);
        wave_order();
        d4 x = mma_xy<LD>(acc_zero(), Ld + r * TT, tmp, -1.0);
        wave_order();
        acc_store<LD>(X + (cc * t + r) * TT, x);
      }
      wave_order();
    }
  }
  return cnt;
}


}  // namespace ahlp
