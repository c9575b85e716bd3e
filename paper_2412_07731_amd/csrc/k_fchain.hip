// Tile path of the Schur-complement factorization and solve (a6) for link
// pairs of at most 16 rows and at most 64 linking variables.
//
// Same segmented elimination as k_chain.hip (segments of consecutive pairs
// eliminated in parallel, then the separator chain, then the x_0 border), but
// every pair block is one 16x16 tile (padded with the identity) and every
// border block a row of t0 = ceil(n0/16) tiles.  A step of the dependent chain
// (factor the current diagonal, form the multipliers, update the next
// diagonal) runs inside one wave with the tile Cholesky of tile_chol.h and
// 16x16x4 MFMAs; the next step's tiles are loaded into registers before the
// current Cholesky.  Everything that does not feed the chain (the separator
// and border updates of a segment, the border sum S00 - sum_k G_k' G_k, the
// separator and border terms of the solve) is computed off the chain, by other
// waves or kernels, and summed in a fixed order.  In the solve, a segment's
// tiles are first staged in LDS by all four waves so that the chain itself
// only waits on LDS.
//
// Storage (16x16 column-major tiles, per pair k):
//   FLi[k]          inverse of the Cholesky factor of the eliminated diagonal
//   FYn[k]          T[next, k] L_k^-T   (next = k+1, or the right separator)
//   FZ[k]           T[left separator, k] L_k^-T  (interior pairs of segments g > 0)
//   FGt[k][q]       (L_k^-1 E_k)' : t0 tiles, rows x_0, columns pair k
//   FSub[s]         separator chain couplings  T'[s, s-1] L_{s-1}^-T
//   FLb, FLbi       border factor and its inverse, t0 x t0 tiles (r, c) at c*t0 + r
#include "common.h"
#include "kernels.h"
#include "tile_chol.h"

namespace ahlp {

namespace {

constexpr int FT_MAXT0 = 4;     // border tiles (n0 <= 64)
constexpr int FT_MAXSEG = 24;   // longest segment (pairs): its solve tiles fit in LDS
constexpr int FT_SEPSTAGE = 24; // separators whose solve tiles are staged in LDS

#define wsync wave_order

// ---- tile helpers (one wave; tiles column-major, 256 doubles)
struct Op { double v[4]; };   // a tile as an MFMA operand: element 64 s + lane

__device__ __forceinline__ Op op_load(const double* t) {
  const int lane = threadIdx.x & 63;
  Op o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[64 * s + lane];
  return o;
}
__device__ __forceinline__ Op op_zero() {
  Op o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = 0.0;
  return o;
}
// operand of a padded exact column-major block (rows x cols, leading dim ld)
__device__ __forceinline__ Op op_load_exact(const double* src, int rows, int cols, int ld) {
  const int lane = threadIdx.x & 63;
  Op o;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = lane & 15, k = 4 * s + (lane >> 4);
    o.v[s] = (i < rows && k < cols) ? src[i + k * ld] : 0.0;
  }
  return o;
}
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
// padded tile of an exact column-major block; identity on the padded diagonal if diag
__device__ __forceinline__ d4 acc_load_exact(const double* src, int rows, int cols, int ld, bool diag) {
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
// transposed padded tile: element (i, j) = src[j + i*ld]
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
// acc += alpha * X Y'   (X as an operand or a tile, Y a tile)
__device__ __forceinline__ d4 mma_opt(d4 acc, const Op& X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(alpha * X.v[s], Y[64 * s + lane], acc);
  return acc;
}
__device__ __forceinline__ d4 mma_xyt(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(alpha * X[64 * s + lane], Y[64 * s + lane], acc);
  return acc;
}
// acc += alpha * X Y  (Y not transposed: element (k, j) at j*16 + k)
__device__ __forceinline__ d4 mma_xy(d4 acc, const double* X, const double* Y, double alpha) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    acc = mfma(alpha * X[64 * s + lane], Y[(lane & 15) * TS + 4 * s + (lane >> 4)], acc);
  return acc;
}
__device__ __forceinline__ void tile_copy(double* dst, const double* src) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) dst[64 * s + lane] = src[64 * s + lane];
}

// y = X v (X as an operand, v 16 values in LDS): every lane ends with y[lane%16].
__device__ __forceinline__ double op_mv(const Op& X, const double* v) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += X.v[k] * v[4 * k + (lane >> 4)];
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}
// y = X' v: the four partial sums of lane l are y[4 s + l/16] after reducing
// over l%16; returned in lane order y[lane%16] through the 16-value scratch sc.
__device__ __forceinline__ double op_mtv(const Op& X, const double* v, double* sc) {
  const int lane = threadIdx.x & 63;
  const double vi = v[lane & 15];
  double out[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double x = X.v[s] * vi;
    x += __shfl_xor(x, 1);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 8);
    out[s] = x;
  }
  wsync();
  if ((lane & 15) == 0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) sc[4 * s + (lane >> 4)] = out[s];
  }
  wsync();
  const double r = sc[lane & 15];
  wsync();
  return r;
}
__device__ __forceinline__ void vec_put(double* dst, double y) {
  const int lane = threadIdx.x & 63;
  if (lane < 16) dst[lane] = y;
}
__device__ __forceinline__ double vec_get_exact(const double* src, int len) {
  const int i = threadIdx.x & 15;
  return i < len ? src[i] : 0.0;
}

struct FSlot {   // per-segment outputs, tile offsets inside segout
  static constexpr int DIAGL = 0, DIAGR = 256, OFF = 512, ELT = 768;
  static constexpr int ERT = ELT + FT_MAXT0 * 256;
  static constexpr int STRIDE = ERT + FT_MAXT0 * 256;
};
struct FSR {     // per-segment right-hand-side contributions
  static constexpr int DSL = 0, DSR = 16, DS0 = 32;
  static constexpr int STRIDE = 32 + 16 * FT_MAXT0;
};

struct SegMeta {   // pair metadata staged in LDS (pairs lo .. hi of a segment)
  int l[FT_MAXSEG + 2];
  long long tdoff[FT_MAXSEG + 2], tooff[FT_MAXSEG + 2], eoff[FT_MAXSEG + 2], loff[FT_MAXSEG + 2];
  double thr[FT_MAXSEG + 2];
};

__device__ __forceinline__ void meta_load(SegMeta& M, const FChainArgs& c, const long long* loff,
                                          int lo, int hi) {
  for (int k = lo + (int)threadIdx.x; k <= hi; k += blockDim.x) {
    const int t = k - lo;
    M.l[t] = c.l[k];
    M.tdoff[t] = c.tdoff[k];
    M.tooff[t] = k < c.P - 1 ? c.tooff[k] : 0;
    M.eoff[t] = c.eoff[k];
    M.loff[t] = loff ? loff[k] : 0;
    M.thr[t] = c.thrT[k];
  }
}

// copy ntiles tiles (global -> LDS) with all threads of the workgroup
__device__ __forceinline__ void stage_tiles(double* dst, const double* src, int ntiles) {
  for (int i = threadIdx.x; i < ntiles * 256; i += blockDim.x) dst[i] = src[i];
}

}  // namespace

// ----------------------------------------------------------------- factor
__global__ __launch_bounds__(64) void k_fchain_seg_factor(FChainArgs c) {
  __shared__ double cur[256], Li[256], Yn[256], Z[256], ZF[256], xbuf[48];
  __shared__ double Ect[FT_MAXT0 * 256], Gt[FT_MAXT0 * 256];
  __shared__ SegMeta M;
  const int g = blockIdx.x, lane = threadIdx.x;
  const int a = c.seg[g].x, b = c.seg[g].y, t0 = c.t0, n0 = c.n0;
  const bool hasL = g > 0, hasR = g < c.G - 1;
  double* slot = c.segout + (long long)g * FSlot::STRIDE;
  const int lo = hasL ? a - 1 : a, hi = hasR ? b : b - 1;   // metadata index = k - lo
  meta_load(M, c, nullptr, lo, hi);
  __syncthreads();
  {
    const int ta = a - lo, la = M.l[ta];
    acc_store(cur, acc_load_exact(c.Td + M.tdoff[ta], la, la, la, true));
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0)
        acc_store(Ect + q * 256, acc_load_exact_t(c.E + M.eoff[ta] + (long long)16 * q * la,
                                                  min(16, n0 - 16 * q), la, la));
    // T[a-1, a] = T[a, a-1]'
    if (hasL) acc_store(ZF, acc_load_exact_t(c.To + M.tooff[0], M.l[0], la, la));
  }
  __syncthreads();
  int cnt = 0;
  for (int k = a; k < b; ++k) {
    const int t = k - lo, lk = M.l[t];
    const bool more = k + 1 < b;
    const int nxt = more ? k + 1 : (hasR ? b : -1);
    const int ln = nxt >= 0 ? M.l[t + 1] : 0;
    // prefetch: T[nxt, k] as an operand, the next diagonal and border rows
    Op yT = op_zero();
    if (nxt >= 0) yT = op_load_exact(c.To + M.tooff[t], ln, lk, ln);
    d4 nd = {0, 0, 0, 0};
    d4 ne[FT_MAXT0];
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q) ne[q] = d4{0, 0, 0, 0};
    if (more) {
      nd = acc_load_exact(c.Td + M.tdoff[t + 1], ln, ln, ln, true);
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0)
          ne[q] = acc_load_exact_t(c.E + M.eoff[t + 1] + (long long)16 * q * ln,
                                   min(16, n0 - 16 * q), ln, ln);
    }
    cnt += wave_chol_tile<double>(cur, cur, Li, M.thr[t], xbuf);
    tile_copy(c.FLi + (long long)k * 256, Li);
    // Yn = T[nxt,k] L^-T ; Z = ZF L^-T ; Gt = Ect L^-T
    d4 yn = {0, 0, 0, 0}, z = {0, 0, 0, 0};
    d4 gt[FT_MAXT0];
    if (nxt >= 0) yn = mma_opt(yn, yT, Li, 1.0);
    if (hasL) z = mma_xyt(z, ZF, Li, 1.0);
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q) {
      gt[q] = d4{0, 0, 0, 0};
      if (q < t0) gt[q] = mma_xyt(gt[q], Ect + q * 256, Li, 1.0);
    }
    wsync();
    if (nxt >= 0) {
      acc_store(Yn, yn);
      acc_store(c.FYn + (long long)k * 256, yn);
    }
    if (hasL) {
      acc_store(Z, z);
      acc_store(c.FZ + (long long)k * 256, z);
    }
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0) {
        acc_store(Gt + q * 256, gt[q]);
        acc_store(c.FGt + ((long long)k * t0 + q) * 256, gt[q]);
      }
    wsync();
    if (more) {
      nd = mma_xyt(nd, Yn, Yn, -1.0);
      d4 zf = {0, 0, 0, 0};
      if (hasL) zf = mma_xyt(zf, Z, Yn, -1.0);
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) ne[q] = mma_xyt(ne[q], Gt + q * 256, Yn, -1.0);
      acc_store(cur, nd);
      if (hasL) acc_store(ZF, zf);
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) acc_store(Ect + q * 256, ne[q]);
    } else if (hasR) {
      d4 acc = {0, 0, 0, 0};
      acc = mma_xyt(acc, Yn, Yn, -1.0);
      acc_store(slot + FSlot::DIAGR, acc);
      if (hasL) {
        d4 o = {0, 0, 0, 0};
        o = mma_xyt(o, Yn, Z, -1.0);
        acc_store(slot + FSlot::OFF, o);
      }
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) {
          d4 e = {0, 0, 0, 0};
          e = mma_xyt(e, Gt + q * 256, Yn, -1.0);
          acc_store(slot + FSlot::ERT + q * 256, e);
        }
    }
    wsync();
  }
  // left-separator updates, summed in order over the segment
  __syncthreads();
  if (hasL) {
    d4 dd = {0, 0, 0, 0};
    d4 de[FT_MAXT0];
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q) de[q] = d4{0, 0, 0, 0};
    for (int k = a; k < b; ++k) {
      const double* Zk = c.FZ + (long long)k * 256;
      dd = mma_xyt(dd, Zk, Zk, -1.0);
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) de[q] = mma_xyt(de[q], c.FGt + ((long long)k * t0 + q) * 256, Zk, -1.0);
    }
    acc_store(slot + FSlot::DIAGL, dd);
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0) acc_store(slot + FSlot::ELT + q * 256, de[q]);
  }
  if (lane == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// Separator chain (one wave); step s + 1's inputs are loaded during step s.
__global__ __launch_bounds__(64) void k_fchain_sep_factor(FChainArgs c) {
  __shared__ double cur[256], Li[256], Ysub[256], xbuf[48];
  __shared__ double Ect[FT_MAXT0 * 256], Gt[FT_MAXT0 * 256];
  const int S = c.G - 1, t0 = c.t0, n0 = c.n0;
  int cnt = 0;
  // inputs of separator s: reduced diagonal, border rows and coupling to s+1
  auto fetch = [&](int s, d4& dg, d4* ec, Op& off, double& thr) {
    const int p = c.seg[s].y, lp = c.l[p];
    const double* sl = c.segout + (long long)s * FSlot::STRIDE;        // segment s (right sep)
    const double* sr = c.segout + (long long)(s + 1) * FSlot::STRIDE;  // segment s+1 (left sep)
    dg = acc_load_exact(c.Td + c.tdoff[p], lp, lp, lp, true) + acc_load(sl + FSlot::DIAGR) +
         acc_load(sr + FSlot::DIAGL);
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q) {
      ec[q] = d4{0, 0, 0, 0};
      if (q < t0)
        ec[q] = acc_load_exact_t(c.E + c.eoff[p] + (long long)16 * q * lp, min(16, n0 - 16 * q), lp, lp) +
                acc_load(sl + FSlot::ERT + q * 256) + acc_load(sr + FSlot::ELT + q * 256);
    }
    off = (s + 1 < S) ? op_load(sr + FSlot::OFF) : op_zero();
    thr = c.thrT[p];
  };
  d4 dg, ec[FT_MAXT0];
  Op off;
  double thr = 0.0;
  if (S > 0) fetch(0, dg, ec, off, thr);
  for (int s = 0; s < S; ++s) {
    const int p = c.seg[s].y;
    if (s > 0) {
      dg = mma_xyt(dg, Ysub, Ysub, -1.0);
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) ec[q] = mma_xyt(ec[q], Gt + q * 256, Ysub, -1.0);
    }
    wsync();
    acc_store(cur, dg);
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0) acc_store(Ect + q * 256, ec[q]);
    const Op coff = off;
    const double cthr = thr;
    wsync();
    if (s + 1 < S) fetch(s + 1, dg, ec, off, thr);   // in flight during the Cholesky
    cnt += wave_chol_tile<double>(cur, cur, Li, cthr, xbuf);
    tile_copy(c.FLi + (long long)p * 256, Li);
    d4 gt[FT_MAXT0];
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q) {
      gt[q] = d4{0, 0, 0, 0};
      if (q < t0) gt[q] = mma_xyt(gt[q], Ect + q * 256, Li, 1.0);
    }
    d4 ys = {0, 0, 0, 0};
    if (s + 1 < S) ys = mma_opt(ys, coff, Li, 1.0);
    wsync();
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0) {
        acc_store(Gt + q * 256, gt[q]);
        acc_store(c.FGt + ((long long)p * t0 + q) * 256, gt[q]);
      }
    if (s + 1 < S) {
      acc_store(Ysub, ys);
      acc_store(c.FSub + (long long)(s + 1) * 256, ys);
    }
    wsync();
  }
  if (threadIdx.x == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// Partial sums of G_k' G_k over contiguous chunks of pairs (t0 x t0 tiles each).
__global__ __launch_bounds__(64) void k_fchain_s00_partial(FChainArgs c, int chunk) {
  const int t0 = c.t0;
  const int k0 = blockIdx.x * chunk, k1 = min(c.P, k0 + chunk);
  double* out = c.s00part + (long long)blockIdx.x * t0 * t0 * 256;
  for (int q = 0; q < t0; ++q)
    for (int q2 = 0; q2 < t0; ++q2) {
      d4 acc = {0, 0, 0, 0};
      for (int k = k0; k < k1; ++k)
        acc = mma_xyt(acc, c.FGt + ((long long)k * t0 + q) * 256,
                      c.FGt + ((long long)k * t0 + q2) * 256, 1.0);
      acc_store(out + (q * t0 + q2) * 256, acc);
    }
}

// Border: B = -(S00 - sum of the partials) in t0 x t0 tiles (all four waves,
// fixed order), then one wave: blocked Cholesky with tile inverses and the
// block inverse of the factor.
__global__ __launch_bounds__(256) void k_fchain_border(FChainArgs c, int nparts) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n0 = c.n0, t0 = c.t0, lane = threadIdx.x & 63;
  double* B = reinterpret_cast<double*>(smem_raw);   // t0*t0 tiles (r, c) at c*t0 + r
  double* X = B + t0 * t0 * 256;                      // inverse tiles
  double* Ld = X + t0 * t0 * 256;                     // inverted diagonal tiles
  double* tmp = Ld + t0 * 256;
  double* xbuf = tmp + 256;
  __shared__ double s_max;
  for (int idx = threadIdx.x; idx < 256 * t0 * t0; idx += blockDim.x) {
    const int tile = idx / 256, e = idx % 256;
    const int r = tile % t0, cc = tile / t0;
    const int i = 16 * r + (e & 15), j = 16 * cc + (e >> 4);
    double v;
    if (i < n0 && j < n0) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      const double* src = c.s00part + (long long)(r * t0 + cc) * 256 + e;
      const long long stride = (long long)t0 * t0 * 256;
      int pp = 0;
      for (; pp + 4 <= nparts; pp += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += src[(pp + u) * stride];
      }
      for (; pp < nparts; ++pp) acc[0] += src[pp * stride];
      v = -(c.S00[i + j * n0] - ((acc[0] + acc[1]) + (acc[2] + acc[3])));
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    B[idx] = v;
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;   // one wave from here on (wave-scope ordering only)
  if (lane == 0) {
    double md = 0.0;
    for (int i = 0; i < n0; ++i) {
      const int r = i >> 4;
      md = fmax(md, B[(r * t0 + r) * 256 + (i & 15) * 17]);
    }
    s_max = md;
  }
  wsync();
  const double thr = PIVOT_REL * fmax(s_max, 0.0);
  int cnt = 0;
  for (int p = 0; p < t0; ++p) {
    double* Bpp = B + (p * t0 + p) * 256;
    cnt += wave_chol_tile<double>(Bpp, Bpp, Ld + p * 256, thr, xbuf);
    for (int r = p + 1; r < t0; ++r) {
      d4 acc = {0, 0, 0, 0};
      acc = mma_xyt(acc, B + (p * t0 + r) * 256, Ld + p * 256, 1.0);
      wsync();
      acc_store(B + (p * t0 + r) * 256, acc);
    }
    wsync();
    for (int r = p + 1; r < t0; ++r)
      for (int cc = p + 1; cc <= r; ++cc) {
        d4 acc = acc_load(B + (cc * t0 + r) * 256);
        acc = mma_xyt(acc, B + (p * t0 + r) * 256, B + (p * t0 + cc) * 256, -1.0);
        wsync();
        acc_store(B + (cc * t0 + r) * 256, acc);
      }
    wsync();
  }
  // X = L^-1 by block columns
  for (int cc = 0; cc < t0; ++cc) {
    for (int r = 0; r < t0; ++r) {
      if (r < cc) {
        for (int s = 0; s < 4; ++s) X[(cc * t0 + r) * 256 + 64 * s + lane] = 0.0;
      } else if (r == cc) {
        tile_copy(X + (cc * t0 + r) * 256, Ld + r * 256);
      } else {
        d4 acc = {0, 0, 0, 0};
        for (int q = cc; q < r; ++q) acc = mma_xy(acc, B + (q * t0 + r) * 256, X + (cc * t0 + q) * 256, 1.0);
        acc_store(tmp, acc);
        wsync();
        d4 x = {0, 0, 0, 0};
        x = mma_xy(x, Ld + r * 256, tmp, -1.0);
        wsync();
        acc_store(X + (cc * t0 + r) * 256, x);
      }
      wsync();
    }
  }
  for (int idx = lane; idx < 256 * t0 * t0; idx += 64) {
    const int tile = idx / 256;
    const int r = tile % t0, cc = tile / t0;
    c.FLb[idx] = (r >= cc) ? B[idx] : 0.0;
    c.FLbi[idx] = X[idx];
  }
  if (lane == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// ----------------------------------------------------------------- solve
// Forward over a segment (four waves): all waves stage the segment's L^-1 and
// Yn tiles in LDS; wave 0 runs w_k = L_k^-1 (s_k - Yn_{k-1} w_{k-1}); then all
// waves form -sum Z_k w_k (left separator) and -sum G_k' w_k (border) over
// interleaved pairs, combined in wave order; wave 0 adds -Yn_{b-1} w_{b-1}.
__global__ __launch_bounds__(256) void k_fchain_seg_fwd(FChainSolveArgs A) {
  const FChainArgs& c = A.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* stg = reinterpret_cast<double*>(smem_raw);       // 2 tiles per pair: L^-1, Yn
  __shared__ double r[16], wseg[FT_MAXSEG * 16], part[4][16 + 16 * FT_MAXT0];
  __shared__ SegMeta M;
  const int g = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = c.seg[g].x, b = c.seg[g].y, t0 = c.t0, n0 = c.n0, nk = b - a;
  const bool hasL = g > 0, hasR = g < c.G - 1;
  meta_load(M, c, A.loff, a, b - 1);
  for (int i = threadIdx.x; i < nk * 512; i += blockDim.x) {
    const int k = i / 512, e = i % 512;
    stg[i] = (e < 256) ? c.FLi[(long long)(a + k) * 256 + e] : c.FYn[(long long)(a + k) * 256 + e - 256];
  }
  __syncthreads();
  if (wave == 0) {
    double sv = vec_get_exact(A.s + M.loff[0], M.l[0]);
    for (int k = a; k < b; ++k) {
      const int t = k - a;
      const double csv = sv;
      if (k + 1 < b) sv = vec_get_exact(A.s + M.loff[t + 1], M.l[t + 1]);
      double rv = csv;
      if (k > a) rv -= op_mv(op_load(stg + (t - 1) * 512 + 256), wseg + (t - 1) * 16);
      wsync();
      vec_put(r, rv);
      wsync();
      const double w = op_mv(op_load(stg + t * 512), r);
      vec_put(wseg + t * 16, w);
      if (lane < M.l[t]) A.w[M.loff[t] + lane] = w;
      wsync();
    }
  }
  __syncthreads();
  double dl = 0.0, ds[FT_MAXT0] = {0, 0, 0, 0};
  for (int t = wave; t < nk; t += 4) {
    const int k = a + t;
    const double* wv = wseg + t * 16;
    if (hasL) dl -= op_mv(op_load(c.FZ + (long long)k * 256), wv);
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0) ds[q] -= op_mv(op_load(c.FGt + ((long long)k * t0 + q) * 256), wv);
  }
  if (lane < 16) {
    part[wave][lane] = dl;
#pragma unroll
    for (int q = 0; q < FT_MAXT0; ++q)
      if (q < t0) part[wave][16 + 16 * q + lane] = ds[q];
  }
  __syncthreads();
  double* out = A.segrhs + (long long)g * FSR::STRIDE;
  for (int i = threadIdx.x; i < 16 + 16 * t0; i += blockDim.x) {
    const double v = ((part[0][i] + part[1][i]) + (part[2][i] + part[3][i]));
    if (i < 16) out[FSR::DSL + i] = v;
    else if (i - 16 < n0) out[FSR::DS0 + i - 16] = v;
  }
  if (hasR && wave == 0) {
    const int t = nk - 1;
    const double d = op_mv(op_load(c.FYn + (long long)(b - 1) * 256), wseg + t * 16);
    if (lane < 16) out[FSR::DSR + lane] = -d;
  }
}

// Separator chain forward, the border, separator chain backward.  The
// separators' L^-1 and coupling tiles are staged in LDS; the border terms
// -sum G_p' w_p and the backward terms G_p u0 are formed by all four waves.
__global__ __launch_bounds__(256) void k_fchain_sep_solve(FChainSolveArgs A) {
  const FChainArgs& c = A.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* stg = reinterpret_cast<double*>(smem_raw);       // 2 tiles per staged separator
  __shared__ double r[16], sc[16], wsep[FT_SEPSTAGE * 16], csep[FT_SEPSTAGE * 16];
  __shared__ double s0[16 * FT_MAXT0], w0[16 * FT_MAXT0], u0[16 * FT_MAXT0], un[16];
  __shared__ double part[4][16 * FT_MAXT0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = c.G - 1, t0 = c.t0, n0 = c.n0;
  const int nst = S < FT_SEPSTAGE ? S : FT_SEPSTAGE;
  for (int i = threadIdx.x; i < nst * 512; i += blockDim.x) {
    const int s = i / 512, e = i % 512;
    const int p = c.seg[s].y;
    stg[i] = (e < 256) ? c.FLi[(long long)p * 256 + e] : (s > 0 ? c.FSub[(long long)s * 256 + e - 256] : 0.0);
  }
  for (int i = threadIdx.x; i < 16 * t0; i += blockDim.x) {
    double v = 0.0;
    if (i < n0) {
      v = A.s[A.nl + i];
      for (int g = 0; g < c.G; ++g) v += A.segrhs[(long long)g * FSR::STRIDE + FSR::DS0 + i];
    }
    s0[i] = v;
  }
  __syncthreads();
  auto li_tile = [&](int s) -> const double* {
    return s < nst ? stg + s * 512 : c.FLi + (long long)c.seg[s].y * 256;
  };
  auto sub_tile = [&](int s) -> const double* {
    return s < nst ? stg + s * 512 + 256 : c.FSub + (long long)s * 256;
  };
  // forward chain (wave 0); w of the separators kept in LDS (or global past the stage)
  if (wave == 0) {
    for (int s = 0; s < S; ++s) {
      const int p = c.seg[s].y, lp = c.l[p];
      const double* dR = A.segrhs + (long long)s * FSR::STRIDE + FSR::DSR;
      const double* dL = A.segrhs + (long long)(s + 1) * FSR::STRIDE + FSR::DSL;
      double rv = vec_get_exact(A.s + A.loff[p], lp) + dR[lane & 15] + dL[lane & 15];
      if (s > 0) rv -= op_mv(op_load(sub_tile(s)), r);   // r holds w_{s-1}
      wsync();
      vec_put(r, rv);
      wsync();
      const double w = op_mv(op_load(li_tile(s)), r);
      wsync();
      vec_put(r, w);
      if (s < FT_SEPSTAGE) vec_put(wsep + s * 16, w);
      if (lane < lp) A.w[A.loff[p] + lane] = w;
      wsync();
    }
  }
  __syncthreads();
  // border right-hand side: s0 - sum_s G_p' w_p  (four waves, fixed order)
  {
    double acc[FT_MAXT0] = {0, 0, 0, 0};
    for (int s = wave; s < S; s += 4) {
      const int p = c.seg[s].y;
      if (s >= FT_SEPSTAGE) continue;   // separators past the stage are added by wave 0 below
      const double* wv = wsep + s * 16;
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) acc[q] += op_mv(op_load(c.FGt + ((long long)p * t0 + q) * 256), wv);
    }
    if (lane < 16)
#pragma unroll
      for (int q = 0; q < FT_MAXT0; ++q)
        if (q < t0) part[wave][16 * q + lane] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;   // wave 0 only from here
  for (int i = lane; i < 16 * t0; i += 64)
    s0[i] -= ((part[0][i] + part[1][i]) + (part[2][i] + part[3][i]));
  wsync();
  for (int s = FT_SEPSTAGE; s < S; ++s) {   // separators past the stage (rare)
    const int p = c.seg[s].y;
    vec_put(r, vec_get_exact(A.w + A.loff[p], c.l[p]));
    wsync();
    for (int q = 0; q < t0; ++q) {
      const double gq = op_mv(op_load(c.FGt + ((long long)p * t0 + q) * 256), r);
      wsync();
      if (lane < 16) s0[16 * q + lane] -= gq;
      wsync();
    }
  }
  // border: w0 = Lbi s0,  u0 = -Lbi' w0  (lower block-triangular tiles)
  for (int rr = 0; rr < t0; ++rr) {
    double acc = 0.0;
    for (int cc = 0; cc <= rr; ++cc) acc += op_mv(op_load(c.FLbi + (cc * t0 + rr) * 256), s0 + 16 * cc);
    wsync();
    if (lane < 16) w0[16 * rr + lane] = acc;
    wsync();
  }
  for (int cc = 0; cc < t0; ++cc) {
    double acc = 0.0;
    for (int rr = cc; rr < t0; ++rr) acc += op_mtv(op_load(c.FLbi + (cc * t0 + rr) * 256), w0 + 16 * rr, sc);
    if (lane < 16) {
      u0[16 * cc + lane] = -acc;
      if (16 * cc + lane < n0) A.u[A.nl + 16 * cc + lane] = -acc;
    }
    wsync();
  }
  // backward terms c_s = G_p u0 = Gt_p' u0 for the staged separators
  for (int s = 0; s < nst; ++s) {
    const int p = c.seg[s].y;
    double acc = 0.0;
    for (int q = 0; q < t0; ++q) acc += op_mtv(op_load(c.FGt + ((long long)p * t0 + q) * 256), u0 + 16 * q, sc);
    vec_put(csep + s * 16, acc);
  }
  wsync();
  for (int s = S - 1; s >= 0; --s) {
    const int p = c.seg[s].y, lp = c.l[p];
    double rv;
    if (s < FT_SEPSTAGE) {
      rv = wsep[s * 16 + (lane & 15)] - csep[s * 16 + (lane & 15)];
    } else {
      rv = vec_get_exact(A.w + A.loff[p], lp);
      for (int q = 0; q < t0; ++q)
        rv -= op_mtv(op_load(c.FGt + ((long long)p * t0 + q) * 256), u0 + 16 * q, sc);
    }
    if (s + 1 < S) rv -= op_mtv(op_load(sub_tile(s + 1)), un, sc);
    wsync();
    vec_put(r, rv);
    wsync();
    const double u = op_mtv(op_load(li_tile(s)), r, sc);
    if (lane < lp) A.u[A.loff[p] + lane] = u;
    vec_put(un, u);
    wsync();
  }
}

// Backward over a segment (four waves): c_k = Z_k' u_left + G_k u0 for all
// pairs first (interleaved over the waves), the segment's L^-1 and Yn tiles
// staged in LDS, then wave 0 runs u_k = L_k^-T (w_k - Yn_k' u_next - c_k).
__global__ __launch_bounds__(256) void k_fchain_seg_bwd(FChainSolveArgs A) {
  const FChainArgs& c = A.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* stg = reinterpret_cast<double*>(smem_raw);
  __shared__ double r[16], un[16], uL[16], sc[4][16], u0[16 * FT_MAXT0], cseg[FT_MAXSEG * 16];
  __shared__ SegMeta M;
  const int g = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = c.seg[g].x, b = c.seg[g].y, t0 = c.t0, n0 = c.n0, nk = b - a;
  const bool hasL = g > 0, hasR = g < c.G - 1;
  meta_load(M, c, A.loff, a, b - 1);
  for (int i = threadIdx.x; i < 16 * t0; i += blockDim.x) u0[i] = i < n0 ? A.u[A.nl + i] : 0.0;
  if (threadIdx.x < 16) {
    uL[threadIdx.x] = hasL ? vec_get_exact(A.u + A.loff[a - 1], c.l[a - 1]) : 0.0;
    un[threadIdx.x] = hasR ? vec_get_exact(A.u + A.loff[b], c.l[b]) : 0.0;
  }
  for (int i = threadIdx.x; i < nk * 512; i += blockDim.x) {
    const int k = i / 512, e = i % 512;
    stg[i] = (e < 256) ? c.FLi[(long long)(a + k) * 256 + e] : c.FYn[(long long)(a + k) * 256 + e - 256];
  }
  __syncthreads();
  for (int t = wave; t < nk; t += 4) {
    const int k = a + t;
    double acc = 0.0;
    if (hasL) acc += op_mtv(op_load(c.FZ + (long long)k * 256), uL, sc[wave]);
    for (int q = 0; q < t0; ++q)
      acc += op_mtv(op_load(c.FGt + ((long long)k * t0 + q) * 256), u0 + 16 * q, sc[wave]);
    vec_put(cseg + t * 16, acc);
  }
  __syncthreads();
  if (wave != 0) return;
  for (int k = b - 1; k >= a; --k) {
    const int t = k - a, lk = M.l[t];
    double rv = vec_get_exact(A.w + M.loff[t], lk) - cseg[t * 16 + (lane & 15)];
    if (k + 1 < b || hasR) rv -= op_mtv(op_load(stg + t * 512 + 256), un, sc[0]);
    wsync();
    vec_put(r, rv);
    wsync();
    const double u = op_mtv(op_load(stg + t * 512), r, sc[0]);
    if (lane < lk) A.u[M.loff[t] + lane] = u;
    vec_put(un, u);
    wsync();
  }
}

// ------------------------------------------------------------- launchers
bool fchain_supported(int lmax, int n0) { return lmax <= 16 && n0 <= 16 * FT_MAXT0; }
int fchain_seg_stride() { return FSlot::STRIDE; }
int fchain_segrhs_stride() { return FSR::STRIDE; }
int fchain_max_segment() { return FT_MAXSEG; }

static size_t border_smem(int t0) { return (size_t)(2 * t0 * t0 + t0 + 1) * 256 * sizeof(double) + 48 * sizeof(double); }
static size_t segsolve_smem() { return (size_t)FT_MAXSEG * 512 * sizeof(double); }
static size_t sepsolve_smem() { return (size_t)FT_SEPSTAGE * 512 * sizeof(double); }

void launch_fchain_factor(hipStream_t st, const FChainArgs& c, int nparts, int chunk) {
  if (c.G > 0) hipLaunchKernelGGL(k_fchain_seg_factor, dim3(c.G), dim3(64), 0, st, c);
  if (c.G > 1) hipLaunchKernelGGL(k_fchain_sep_factor, dim3(1), dim3(64), 0, st, c);
  if (c.n0 > 0) {
    if (nparts > 0)
      hipLaunchKernelGGL(k_fchain_s00_partial, dim3(nparts), dim3(64), 0, st, c, chunk);
    hipLaunchKernelGGL(k_fchain_border, dim3(1), dim3(256), border_smem(c.t0), st, c, nparts);
  }
}

void launch_fchain_solve(hipStream_t st, const FChainSolveArgs& a) {
  if (a.c.G > 0) hipLaunchKernelGGL(k_fchain_seg_fwd, dim3(a.c.G), dim3(256), segsolve_smem(), st, a);
  hipLaunchKernelGGL(k_fchain_sep_solve, dim3(1), dim3(256), sepsolve_smem(), st, a);
  if (a.c.G > 0) hipLaunchKernelGGL(k_fchain_seg_bwd, dim3(a.c.G), dim3(256), segsolve_smem(), st, a);
}

void set_fchain_smem_limits(size_t) {
  hipFuncSetAttribute((const void*)k_fchain_border, hipFuncAttributeMaxDynamicSharedMemorySize, (int)border_smem(FT_MAXT0));
  hipFuncSetAttribute((const void*)k_fchain_seg_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)segsolve_smem());
  hipFuncSetAttribute((const void*)k_fchain_seg_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)segsolve_smem());
  hipFuncSetAttribute((const void*)k_fchain_sep_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sepsolve_smem());
}

}  // namespace ahlp
