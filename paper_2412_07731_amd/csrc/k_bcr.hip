// Block cyclic reduction of the Schur complement (a6) for link pairs of at
// most 16 rows and at most 64 linking variables (pairs of up to 32 rows:
// k_bcr2.hip, which shares the border kernels below).
//
// The assembled Schur complement is S = [T E; E' S00] with T block
// tridiagonal over the P link pairs (App. A) and E, S00 the x_0 border.  T is
// eliminated by odd-even reduction: at level v the active pairs are
// j = k 2^v (k = 0 .. n_v - 1); the pairs at odd positions k are eliminated
// all at once (each is coupled only to its two active neighbours), which
// updates the even ones and couples neighbouring even pairs; the evens form
// level v + 1.  This is the elimination of Alg. 3 of the Schur solve in a
// symmetric permutation of T that turns its dependent chain of P steps into
// ceil(log2 P) levels of independent steps.  For an eliminated pair o with
// active neighbours L (left) and R (right):
//   T'_oo = L_o L_o',  X_L = L_o^-1 T'_oL,  X_R = L_o^-1 T'_oR,  Z = L_o^-1 E'_o
//   T'_LL -= X_L'X_L,  T'_RR -= X_R'X_R,  T'_RL = -X_R'X_L,
//   E'_L -= X_L'Z,  E'_R -= X_R'Z,  S00 - sum over all pairs of Z'Z.
// The border Schur complement S00 - E'T^-1 E is negative definite (the
// system is quasi-definite) and is factorized as -(S00 - sum Z'Z) = Lb Lb'.
//
// Storage: 16x16 column-major tiles per pair j, padded with the identity.
//   BD[j], BC[j], BEt[j][q]   working diagonal, coupling T'[next active, j]
//                             and border rows (transposed, t0 tiles)
//   FLi[o], FXL[o], FXR[o]    L_o^-1, X_L, X_R of the eliminated pair o
//   FGt[o][q]                 Z' of pair o (t0 tiles), the final pair included
//   FLb, FLbi                 border factor and its inverse, tiles (r, c) at c*t0 + r
// Wide levels (more than TAIL_WAVES eliminations) run as one launch per level
// (factor: both eliminations next to an even pair and its update in one
// workgroup); the narrow levels, the final pair and (in the solve) the border
// run inside one workgroup.  Every sum is taken in a fixed order.
#include "common.h"
#include "kernels.h"
#include "tile_chol.h"
#include "tile_ops.h"
#include "bcr_border.h"

namespace ahlp {

namespace {

constexpr int BT_MAXT0 = 4;      // border tiles (n0 <= 64)
constexpr int TAIL_WAVES = 8;    // waves of the single-workgroup factor tail
constexpr int TAIL_WAVES_S = 16; // waves of the single-workgroup solve tail
// LDS tiles of the eliminating kernels are column-major with leading
// dimension 17: accumulator-layout writes and B-operand reads walk a tile by
// columns across the lanes, which with 16 would put 16 lanes in one bank
constexpr int PLD = TS + 1, PTE = TS * PLD;
constexpr int ELIM_LDS = 2 * PTE;   // doubles of LDS per eliminating wave: the tile, L^-1

// ---------------------------------------------------------------- factor
// Working tiles from the assembled parts (one wave per tile).
__global__ __launch_bounds__(256) void k_bcr_init(BcrArgs c) {
  const int per = 2 + c.t0;
  const long long wt = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wt >= (long long)c.P * per) return;
  const int j = (int)(wt / per), kind = (int)(wt % per), lj = c.l[j];
  if (kind == 0) {
    acc_store(c.BD + (long long)j * 256, acc_load_exact(c.Td + c.tdoff[j], lj, lj, lj, true));
  } else if (kind == 1) {
    if (j + 1 < c.P) {
      const int ln = c.l[j + 1];
      acc_store(c.BC + (long long)j * 256, acc_load_exact(c.To + c.tooff[j], ln, lj, ln, false));
    }
  } else {
    const int q = kind - 2;
    acc_store(c.BEt + ((long long)j * c.t0 + q) * 256,
              acc_load_exact_t(c.E + c.eoff[j] + 16LL * q * lj, min(16, c.n0 - 16 * q), lj, lj));
  }
}

// Tile operands in registers: ld_a(X) gives X as the A operand of X*Y or
// X*Y' (and Y as the B operand of X*Y'); ld_b(X) gives X as the B operand of
// Y*X or the A/B operand of X'*Y.  All operands of a step are loaded before
// any of them is used, so a step waits on memory once.
struct T4 { double v[4]; };
__device__ __forceinline__ T4 ld_a(const double* __restrict__ t) {
  const int lane = threadIdx.x & 63;
  T4 o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[64 * s + lane];
  return o;
}
__device__ __forceinline__ T4 ld_b(const double* __restrict__ t) {
  const int lane = threadIdx.x & 63;
  const int idx = (lane & 15) * TS + (lane >> 4);
  T4 o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[idx + 4 * s];
  return o;
}
__device__ __forceinline__ T4 t4_zero() { return T4{{0.0, 0.0, 0.0, 0.0}}; }
// the same operations on padded LDS tiles (element col 16 + row at col 17 + row)
__device__ __forceinline__ int pe(int e) { return e + (e >> 4); }
__device__ __forceinline__ void acc_store_l(double* t, const d4& a) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[pe(acc_index<double>(lane, r))] = a[r];
}
__device__ __forceinline__ T4 ld_a_l(const double* t) {
  const int lane = threadIdx.x & 63;
  T4 o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[pe(64 * s + lane)];
  return o;
}
__device__ __forceinline__ T4 ld_b_l(const double* t) {
  const int lane = threadIdx.x & 63;
  const int idx = (lane & 15) * TS + (lane >> 4);
  T4 o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[pe(idx + 4 * s)];
  return o;
}
__device__ __forceinline__ void tile_copy_l(double* __restrict__ dst, const double* src) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) dst[64 * s + lane] = src[pe(64 * s + lane)];
}
// acc + alpha * (product with the given operands)
__device__ __forceinline__ d4 mm(d4 acc, const T4& a, const T4& b, double alpha) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(alpha * a.v[s], b.v[s], acc);
  return acc;
}

// Eliminate pair o (active neighbours L if needXL, R if hasR): factor its
// working diagonal and form X_L = L_o^-1 T'[o,L], X_R = L_o^-1 T'[R,o]' and
// G_q = (L_o^-1 E'_o)' (accumulator layout).  scr: ELIM_LDS doubles of this
// wave; L_o^-1 is left in scr + PTE (padded).  Returns replaced pivots.
__device__ int elim_core(const BcrArgs& c, long long o, long long L, bool needXL, bool hasR,
                         double* scr, d4& XL, d4& XR, d4* G) {
  double* cur = scr;
  double* Li = scr + PTE;
  const double* __restrict__ BC = c.BC;
  const double* __restrict__ BEt = c.BEt;
  const d4 D = acc_load(c.BD + o * 256);
  const double thr = c.thrT[o];
  T4 cl = t4_zero(), cr = t4_zero(), et[BT_MAXT0];
  if (needXL) cl = ld_b(BC + L * 256);
  if (hasR) cr = ld_a(BC + o * 256);
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q) et[q] = q < c.t0 ? ld_a(BEt + (o * c.t0 + q) * 256) : t4_zero();
  acc_store_l(cur, D);
  wave_order();
  const int cnt = wave_chol_tile<double, PLD>(cur, cur, Li, thr, nullptr);
  const T4 li = ld_a_l(Li);
  XL = needXL ? mm(acc_zero(), li, cl, 1.0) : acc_zero();
  XR = hasR ? mm(acc_zero(), li, cr, 1.0) : acc_zero();
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q) G[q] = q < c.t0 ? mm(acc_zero(), et[q], li, 1.0) : acc_zero();
  return cnt;
}

// store the factor of pair o (L^-1 from its padded LDS tile)
__device__ void store_factor(const BcrArgs& c, long long o, const double* Li, const d4& XL,
                             const d4& XR, bool hasR, const d4* G) {
  tile_copy_l(c.FLi + o * 256, Li);
  acc_store(c.FXL + o * 256, XL);
  if (hasR) acc_store(c.FXR + o * 256, XR);
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q)
    if (q < c.t0) acc_store(c.FGt + (o * c.t0 + q) * 256, G[q]);
}

// One wide level (n active pairs): a workgroup of two waves per even position
// k.  Wave 0 eliminates the right neighbour o_r (and stores its factor: every
// odd pair has exactly one left neighbour), wave 1 eliminates the left one
// o_l again; both leave their products in LDS and the update of the even pair
// is split: wave 0 the diagonal and the new coupling, wave 1 the border rows.
__global__ __launch_bounds__(128) void k_bcr_level(BcrArgs c, int lvl, int n) {
  __shared__ double scr[2][ELIM_LDS];
  __shared__ double xr_[2][(2 + BT_MAXT0) * PTE];   // per wave: X_L, X_R, G_q (padded)
  const int wave = threadIdx.x >> 6, k = 2 * blockIdx.x;
  const long long s = 1LL << lvl, e = k * s;
  const bool hl = k >= 1, hr = k + 1 < n, hrr = k + 2 < n;
  int cnt = 0;
  // the even pair's own tiles, loaded before the elimination
  d4 Dp = acc_zero(), etp[BT_MAXT0];
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q) etp[q] = acc_zero();
  if (wave == 0) {
    Dp = acc_load(c.BD + e * 256);
  } else {
#pragma unroll
    for (int q = 0; q < BT_MAXT0; ++q)
      if (q < c.t0) etp[q] = acc_load(c.BEt + (e * c.t0 + q) * 256);
  }
  const bool mine = wave == 0 ? hr : hl;
  if (mine) {
    d4 XL, XR, G[BT_MAXT0];
    const long long o = wave == 0 ? (k + 1) * s : (k - 1) * s;
    const bool needXL = wave == 0, hasR = wave == 0 ? hrr : true;
    cnt = elim_core(c, o, e, needXL, hasR, scr[wave], XL, XR, G);
    double* x = xr_[wave];
    acc_store_l(x, XL);
    acc_store_l(x + PTE, XR);
#pragma unroll
    for (int q = 0; q < BT_MAXT0; ++q)
      if (q < c.t0) acc_store_l(x + (2 + q) * PTE, G[q]);
    if (wave == 0) store_factor(c, o, scr[0] + PTE, XL, XR, hasR, G);
  }
  __syncthreads();
  const double* xo = xr_[0];   // products of o_r
  const double* xl = xr_[1];   // products of o_l
  if (wave == 0) {
    d4 D = Dp;
    const T4 a = hl ? ld_b_l(xl + PTE) : t4_zero();   // X_R(o_l)
    const T4 b = hr ? ld_b_l(xo) : t4_zero();         // X_L(o_r)
    if (hl) D = mm(D, a, a, -1.0);
    if (hr) D = mm(D, b, b, -1.0);
    acc_store(c.BD + e * 256, D);
    if (hr && hrr) acc_store(c.BC + e * 256, mm(acc_zero(), ld_b_l(xo + PTE), b, -1.0));
  } else {
    d4 et[BT_MAXT0];
#pragma unroll
    for (int q = 0; q < BT_MAXT0; ++q) et[q] = etp[q];
    const T4 a = hl ? ld_b_l(xl + PTE) : t4_zero();
    const T4 b = hr ? ld_b_l(xo) : t4_zero();
#pragma unroll
    for (int q = 0; q < BT_MAXT0; ++q)
      if (q < c.t0) {
        if (hl) et[q] = mm(et[q], ld_a_l(xl + (2 + q) * PTE), a, -1.0);
        if (hr) et[q] = mm(et[q], ld_a_l(xo + (2 + q) * PTE), b, -1.0);
        acc_store(c.BEt + (e * c.t0 + q) * 256, et[q]);
      }
  }
  // o_l is also the right neighbour of the even pair k - 2: its pivots are
  // counted there
  if (threadIdx.x == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// Narrow levels from lvl (n active pairs) down to one pair, then the final
// pair; one workgroup of TAIL_WAVES waves: odd pairs eliminated (factor
// stored), barrier, even pairs updated from the stored products, barrier.
__global__ __launch_bounds__(64 * TAIL_WAVES) void k_bcr_tail(BcrArgs c, int lvl, int n) {
  __shared__ double scr[TAIL_WAVES][ELIM_LDS];
  const int wave = threadIdx.x >> 6;
  int cnt = 0;
  for (; n > 1; ++lvl, n = (n + 1) / 2) {
    const long long s = 1LL << lvl;
    for (int w = wave; w < n / 2; w += TAIL_WAVES) {
      const int k = 2 * w + 1;
      const bool hasR = k + 1 < n;
      d4 XL, XR, G[BT_MAXT0];
      cnt += elim_core(c, k * s, (k - 1) * s, true, hasR, scr[wave], XL, XR, G);
      store_factor(c, k * s, scr[wave] + PTE, XL, XR, hasR, G);
      wave_order();
    }
    __syncthreads();
    for (int w = wave; w < (n + 1) / 2; w += TAIL_WAVES) {
      const int k = 2 * w;
      const long long e = k * s, ol = (k - 1) * s, orr = (k + 1) * s;
      const bool hl = k >= 1, hr = k + 1 < n, hrr = k + 2 < n;
      const double* __restrict__ FXL = c.FXL;
      const double* __restrict__ FXR = c.FXR;
      const double* __restrict__ FGt = c.FGt;
      d4 D = acc_load(c.BD + e * 256);
      const T4 a = hl ? ld_b(FXR + ol * 256) : t4_zero();
      const T4 b = hr ? ld_b(FXL + orr * 256) : t4_zero();
      const T4 xrr = (hr && hrr) ? ld_b(FXR + orr * 256) : t4_zero();
      d4 et[BT_MAXT0];
      T4 gl[BT_MAXT0], gr[BT_MAXT0];
#pragma unroll
      for (int q = 0; q < BT_MAXT0; ++q) {
        const bool on = q < c.t0;
        et[q] = on ? acc_load(c.BEt + (e * c.t0 + q) * 256) : acc_zero();
        gl[q] = (on && hl) ? ld_a(FGt + (ol * c.t0 + q) * 256) : t4_zero();
        gr[q] = (on && hr) ? ld_a(FGt + (orr * c.t0 + q) * 256) : t4_zero();
      }
      if (hl) D = mm(D, a, a, -1.0);
      if (hr) D = mm(D, b, b, -1.0);
      acc_store(c.BD + e * 256, D);
      if (hr && hrr) acc_store(c.BC + e * 256, mm(acc_zero(), xrr, b, -1.0));
#pragma unroll
      for (int q = 0; q < BT_MAXT0; ++q)
        if (q < c.t0) {
          if (hl) et[q] = mm(et[q], gl[q], a, -1.0);
          if (hr) et[q] = mm(et[q], gr[q], b, -1.0);
          acc_store(c.BEt + (e * c.t0 + q) * 256, et[q]);
        }
    }
    __syncthreads();
  }
  if (n == 1 && wave == 0) {
    d4 XL, XR, G[BT_MAXT0];
    cnt += elim_core(c, 0, 0, false, false, scr[0], XL, XR, G);
    tile_copy_l(c.FLi, scr[0] + PTE);
#pragma unroll
    for (int q = 0; q < BT_MAXT0; ++q)
      if (q < c.t0) acc_store(c.FGt + q * 256, G[q]);
  }
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// Partial sums of Z_j'Z_j = FGt_j FGt_j' over contiguous chunks of pairs, one
// wave per (chunk, border tile (q, q2)).  Pair j's tile (q, c) of FGt is at
// (j tp + c) t0 + q, so u = j tp + c runs over a chunk's tiles in order.
__global__ __launch_bounds__(64) void k_bcr_s00_partial(BcrArgs c, int chunk) {
  const int t0 = c.t0, tp = c.tp, nt = t0 * t0;
  const int part = blockIdx.x / nt, t = blockIdx.x % nt, q = t / t0, q2 = t % t0;
  const long long u0 = (long long)part * chunk * tp;
  const long long u1 = (long long)min(c.P, (part + 1) * chunk) * tp;
  const double* __restrict__ G = c.FGt;
  d4 acc = acc_zero();
#pragma unroll 4
  for (long long u = u0; u < u1; ++u)
    acc = mma_xyt(acc, G + (u * t0 + q) * 256, G + (u * t0 + q2) * 256, 1.0);
  acc_store(c.s00part + ((long long)part * nt + t) * 256, acc);
}

// Sum of the chunk partials, one thread per element, chunks in order; the
// sum goes after the nparts partials.
__global__ __launch_bounds__(256) void k_bcr_s00_sum(BcrArgs c, int nparts) {
  const int n = c.t0 * c.t0 * 256;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const double* src = c.s00part + idx;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int pp = 0;
#pragma unroll 4
  for (; pp + 4 <= nparts; pp += 4)
    for (int u = 0; u < 4; ++u) acc[u] += src[(long long)(pp + u) * n];
  for (; pp < nparts; ++pp) acc[0] += src[(long long)pp * n];
  c.s00part[(long long)nparts * n + idx] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Border: B = -(S00 - sum of Z_j'Z_j) in t0 x t0 tiles (all four waves), then
// one wave: blocked Cholesky with tile inverses and the block inverse of the
// factor.  With global rows in the border (c.ng > 0) B is quasi-definite
// (negative definite on the global rows, positive on x_0) and the
// factorization is the signed one, B = Lb T Lb' with T = diag(-I, I).
__global__ __launch_bounds__(256) void k_bcr_border(BcrArgs c, int nparts) {
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
      const double zz = nparts > 0 ? c.s00part[((long long)nparts * t0 * t0 + r * t0 + cc) * 256 + e] : 0.0;
      v = -(c.S00[i + j * n0] - zz);
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
      md = fmax(md, fabs(B[(r * t0 + r) * 256 + (i & 15) * 17]));
    }
    s_max = md;
  }
  wave_order();
  const double thr = PIVOT_REL * s_max;
  // the global rows' part of B is negative definite: signed factorization there
  const unsigned long long neg = c.ng >= 64 ? ~0ull : ((1ull << c.ng) - 1ull);
  const int cnt = wave_block_chol(B, t0, X, Ld, tmp, xbuf, thr, neg);
  for (int idx = lane; idx < 256 * t0 * t0; idx += 64) {
    const int tile = idx / 256;
    const int r = tile % t0, cc = tile / t0;
    c.FLb[idx] = (r >= cc) ? B[idx] : 0.0;
    c.FLbi[idx] = X[idx];
  }
  if (lane == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// ----------------------------------------------------------------- solve
// Forward: r_e -= X_R(o_l)' w_{o_l} + X_L(o_r)' w_{o_r} with w_o = L_o^-1 r_o;
// backward: u_o = L_o^-T (w_o - X_L u_L - X_R u_R - Z_o u0).  The pair vectors
// r, w, u are padded to 16 per pair; level 0 reads the exact right-hand side.
// The wide levels keep them in the global arrays r, w, up; the single-workgroup
// tail keeps the vectors of its pairs (every 2^lt-th pair, lt its first level)
// in LDS, slot j >> lt, and writes to global memory only what later launches
// read: u (and up for the wide backward levels) and the border partials.
struct VecLds { double v0[16], v1[16], sc[16], ua[16], ub[16]; };
constexpr int TAIL_SLOTS = 2 * TAIL_WAVES_S + 2;   // pairs at the tail's first level, at most
struct TailVecs { double r[TAIL_SLOTS * 16], w[TAIL_SLOTS * 16], u[TAIL_SLOTS * 16]; };
// where the pair vectors of one level live: T == nullptr for a wide level,
// else the tail's LDS with r read from the global arrays at its first level
struct VecPlace {
  TailVecs* T;
  int shift;     // slot = position << shift at this level
  bool r_lds;    // r of this level in LDS (not the tail's first level)
};

__device__ __forceinline__ double rvec(const BcrSolveArgs& A, int lvl, long long j) {
  if (lvl == 0) return vec_get_exact(A.s + A.loff[j], A.c.l[j]);
  return A.r[j * 16 + (threadIdx.x & 15)];
}
__device__ __forceinline__ double rget(const BcrSolveArgs& A, const VecPlace& P, int lvl, int k) {
  if (P.r_lds) return P.T->r[(k << P.shift) * 16 + (threadIdx.x & 15)];
  return rvec(A, lvl, (long long)k << lvl);
}

// even position k of level lvl: updates r_e; stores w and the border
// partial Z'w of its right neighbour (each odd pair has exactly one left one).
// All loads of the step are issued first.
__device__ void bcr_fwd_even(const BcrSolveArgs& A, int lvl, int n, int k, VecLds& V,
                             const VecPlace& P) {
  const BcrArgs& c = A.c;
  const int lane = threadIdx.x & 63;
  const long long s = 1LL << lvl, e = k * s, ol = (k - 1) * s, orr = (k + 1) * s;
  const bool hl = k >= 1, hr = k + 1 < n;
  const double re = rget(A, P, lvl, k);
  const double rl = hl ? rget(A, P, lvl, k - 1) : 0.0;
  const double rr = hr ? rget(A, P, lvl, k + 1) : 0.0;
  Op lil{}, xrl{}, lir{}, xlr{}, g[BT_MAXT0];
  if (hl) {
    lil = op_load(c.FLi + ol * 256);
    xrl = op_load(c.FXR + ol * 256);
  }
  if (hr) {
    lir = op_load(c.FLi + orr * 256);
    xlr = op_load(c.FXL + orr * 256);
  }
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q)
    if (hr && q < c.t0) g[q] = op_load(c.FGt + (orr * c.t0 + q) * 256);
  vec_put(V.v0, rl);
  vec_put(V.ua, rr);
  wave_order();
  const double wl = hl ? op_mv(lil, V.v0) : 0.0;
  const double wr = hr ? op_mv(lir, V.ua) : 0.0;
  vec_put(V.v1, wl);
  vec_put(V.ub, wr);
  wave_order();
  double acc = re;
  if (hl) acc -= op_mtv(xrl, V.v1, V.sc);
  if (hr) {
    acc -= op_mtv(xlr, V.ub, V.sc);
    if (lane < 16) {
      if (P.T) P.T->w[((k + 1) << P.shift) * 16 + lane] = wr;
      else A.w[orr * 16 + lane] = wr;
    }
#pragma unroll
    for (int q = 0; q < BT_MAXT0; ++q)
      if (q < c.t0) {
        const double pq = op_mv(g[q], V.ub);
        if (lane < 16) A.pb[(orr * c.t0 + q) * 16 + lane] = pq;
      }
  }
  wave_order();
  if (lane < 16) {
    if (P.T) P.T->r[(k << P.shift) * 16 + lane] = acc;
    else A.r[e * 16 + lane] = acc;
  }
}

// the final pair (j = 0) forward: w_0 (to the tail's slot 0) and its border
// partial
__device__ void bcr_final_fwd(const BcrSolveArgs& A, int lvl, VecLds& V, const VecPlace& P) {
  const BcrArgs& c = A.c;
  const int lane = threadIdx.x & 63;
  const double r0 = rget(A, P, lvl, 0);
  const Op li = op_load(c.FLi);
  Op g[BT_MAXT0];
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q)
    if (q < c.t0) g[q] = op_load(c.FGt + q * 256);
  vec_put(V.v0, r0);
  wave_order();
  const double w = op_mv(li, V.v0);
  vec_put(V.v1, w);
  wave_order();
  if (lane < 16) P.T->w[lane] = w;
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q)
    if (q < c.t0) {
      const double pq = op_mv(g[q], V.v1);
      if (lane < 16) A.pb[q * 16 + lane] = pq;
    }
  wave_order();
}

// u_o of odd position k of level lvl (n positions) from w_o, the neighbours'
// u and u0; k = 0, n = 1: the final pair
__device__ void bcr_bwd_pair(const BcrSolveArgs& A, int lvl, int n, int k, const double* u0,
                             VecLds& V, const VecPlace& P) {
  const BcrArgs& c = A.c;
  const int lane = threadIdx.x & 63, i16 = lane & 15;
  const long long s = 1LL << lvl, o = k * s, L = (k - 1) * s, R = (k + 1) * s;
  const bool hl = k >= 1, hr = k + 1 < n;
  double wv, ul = 0.0, ur = 0.0;
  if (P.T) {
    wv = P.T->w[(k << P.shift) * 16 + i16];
    if (hl) ul = P.T->u[((k - 1) << P.shift) * 16 + i16];
    if (hr) ur = P.T->u[((k + 1) << P.shift) * 16 + i16];
  } else {
    wv = A.w[o * 16 + i16];
    if (hl) ul = A.up[L * 16 + i16];
    if (hr) ur = A.up[R * 16 + i16];
  }
  Op xl{}, xr{}, g[BT_MAXT0];
  if (hl) xl = op_load(c.FXL + o * 256);
  if (hr) xr = op_load(c.FXR + o * 256);
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q)
    if (q < c.t0) g[q] = op_load(c.FGt + (o * c.t0 + q) * 256);
  const Op li = op_load(c.FLi + o * 256);
  vec_put(V.ua, ul);
  vec_put(V.ub, ur);
  wave_order();
  double v = wv;
  if (hl) v -= op_mv(xl, V.ua);
  if (hr) v -= op_mv(xr, V.ub);
#pragma unroll
  for (int q = 0; q < BT_MAXT0; ++q)
    if (q < c.t0) v -= op_mtv(g[q], u0 + 16 * q, V.sc);
  vec_put(V.v1, v);
  wave_order();
  const double u = op_mtv(li, V.v1, V.sc);
  if (lane < 16) {
    A.up[o * 16 + lane] = u;
    if (P.T) P.T->u[(k << P.shift) * 16 + lane] = u;
  }
  if (lane < c.l[o]) A.u[A.loff[o] + lane] = u;
  wave_order();
}

__global__ __launch_bounds__(256) void k_bcr_fwd(BcrSolveArgs A, int lvl, int n) {
  __shared__ VecLds V[4];
  const int wave = threadIdx.x >> 6, w = blockIdx.x * 4 + wave;
  if (w >= (n + 1) / 2) return;
  bcr_fwd_even(A, lvl, n, 2 * w, V[wave], VecPlace{nullptr, 0, false});
}

__global__ __launch_bounds__(256) void k_bcr_bwd(BcrSolveArgs A, int lvl, int n) {
  __shared__ VecLds V[4];
  __shared__ double u0[16 * BT_MAXT0];
  const int wave = threadIdx.x >> 6, w = blockIdx.x * 4 + wave;
  for (int i = threadIdx.x; i < 16 * A.c.t0; i += blockDim.x) u0[i] = A.u0p[i];
  __syncthreads();
  if (w >= n / 2) return;
  bcr_bwd_pair(A, lvl, n, 2 * w + 1, u0, V[wave], VecPlace{nullptr, 0, false});
}

// lower triangle of the border factor's Lb^-1 tiles into LDS, packed (tile
// (r, c) at r (r + 1) / 2 + c), by the threads first .. first + count - 1
__device__ void stage_lbi(const BcrArgs& c, double* lbi, int first, int count) {
  const int t0 = c.t0;
  for (int idx = threadIdx.x - first; idx < t0 * (t0 + 1) / 2 * 256; idx += count) {
    const int tile = idx >> 8, e = idx & 255;
    int r = 0;
    while ((r + 1) * (r + 2) / 2 <= tile) ++r;
    const int cc = tile - r * (r + 1) / 2;
    lbi[idx] = c.FLbi[(cc * t0 + r) * 256 + e];
  }
}

// Narrow forward levels from lvl (n active pairs), the final pair, the border
// right-hand side s0 - sum_j Z_j'w_j (fixed order), the border solve
// w0 = Lb^-1 s0, u0 = -Lb^-T w0, the final pair backward and the narrow
// backward levels.  One workgroup of TAIL_WAVES_S waves; the levels are
// separated by LDS-only barriers, since the pair vectors stay in LDS.  The
// Lb^-1 tiles are staged in LDS by the waves left idle at the second level.
__global__ __launch_bounds__(64 * TAIL_WAVES_S) void k_bcr_tail_solve(BcrSolveArgs A, int lvl, int n) {
  const BcrArgs& c = A.c;
  __shared__ VecLds V[TAIL_WAVES_S];
  __shared__ TailVecs T;
  __shared__ double lbi[BT_MAXT0 * (BT_MAXT0 + 1) / 2 * 256];
  __shared__ double part[64 * TAIL_WAVES_S];
  __shared__ double s0[16 * BT_MAXT0], w0[16 * BT_MAXT0], u0[16 * BT_MAXT0];
  __shared__ int lv_n[32];
  const int wave = threadIdx.x >> 6;
  const int lt = lvl;
  int nlev = 0;
  bool staged = false;
  for (; n > 1; ++lvl, n = (n + 1) / 2) {
    const int ne = (n + 1) / 2;
    if (threadIdx.x == 0) lv_n[nlev] = n;
    if (nlev == 1 && ne < TAIL_WAVES_S) {
      if (wave >= ne) stage_lbi(c, lbi, 64 * ne, 64 * (TAIL_WAVES_S - ne));
      staged = true;
    }
    const VecPlace P{&T, lvl - lt, lvl > lt};
    for (int w = wave; w < ne; w += TAIL_WAVES_S) bcr_fwd_even(A, lvl, n, 2 * w, V[wave], P);
    ++nlev;
    lds_barrier();
  }
  if (!staged) stage_lbi(c, lbi, 0, blockDim.x);
  if (n == 1 && wave == 0) bcr_final_fwd(A, lvl, V[0], VecPlace{&T, lvl - lt, lvl > lt});
  // full barrier: the border sum reads the partials stored to global memory
  __syncthreads();
  bcr_border_solve(A, lbi, true, part, s0, w0, u0, V[0].sc);
  if (c.P >= 1 && wave == 0) bcr_bwd_pair(A, lvl, 1, 0, u0, V[0], VecPlace{&T, lvl - lt, true});
  lds_barrier();
  for (int li = nlev - 1; li >= 0; --li) {
    const int nn = lv_n[li], lv = lt + li;
    const VecPlace P{&T, li, true};
    for (int w = wave; w < nn / 2; w += TAIL_WAVES_S) bcr_bwd_pair(A, lv, nn, 2 * w + 1, u0, V[wave], P);
    lds_barrier();
  }
}

size_t border_smem(int t0) {
  return (size_t)(2 * t0 * t0 + t0 + 1) * 256 * sizeof(double) + 48 * sizeof(double);
}

// first level handled by a tail kernel of `waves` waves: the first with at
// most that many eliminations
int tail_level(int P, int waves, int* n_out) {
  int lvl = 0, n = P;
  while (n > 1 && n / 2 > waves) {
    ++lvl;
    n = (n + 1) / 2;
  }
  *n_out = n;
  return lvl;
}

}  // namespace

int bcr_tiles(int lmax, int n0) {
  if (n0 > 16 * BT_MAXT0) return 0;
  return lmax <= 16 ? 1 : lmax <= 32 ? 2 : 0;
}

void launch_bcr_factor(hipStream_t st, const BcrArgs& c, int nparts, int chunk) {
  if (c.tp == 2) {
    launch_bcr2_reduce(st, c);
  } else if (c.P > 0) {
    const long long tiles = (long long)c.P * (2 + c.t0);
    hipLaunchKernelGGL(k_bcr_init, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, c);
    int nt = 0;
    const int lt = tail_level(c.P, TAIL_WAVES, &nt);
    int n = c.P;
    for (int lvl = 0; lvl < lt; ++lvl, n = (n + 1) / 2)
      hipLaunchKernelGGL(k_bcr_level, dim3((n + 1) / 2), dim3(128), 0, st, c, lvl, n);
    hipLaunchKernelGGL(k_bcr_tail, dim3(1), dim3(64 * TAIL_WAVES), 0, st, c, lt, nt);
  }
  if (c.n0 > 0) {
    if (nparts > 0) {
      hipLaunchKernelGGL(k_bcr_s00_partial, dim3(nparts * c.t0 * c.t0), dim3(64), 0, st, c, chunk);
      hipLaunchKernelGGL(k_bcr_s00_sum, dim3((c.t0 * c.t0 * 256 + 255) / 256), dim3(256), 0, st, c, nparts);
    }
    hipLaunchKernelGGL(k_bcr_border, dim3(1), dim3(256), border_smem(c.t0), st, c, nparts);
  }
}

void launch_bcr_solve(hipStream_t st, const BcrSolveArgs& a) {
  if (a.c.tp == 2) {
    launch_bcr2_solve(st, a);
    return;
  }
  const int P = a.c.P;
  int nt = 0;
  const int lt = P > 0 ? tail_level(P, TAIL_WAVES_S, &nt) : 0;
  int n = P;
  for (int lvl = 0; lvl < lt; ++lvl, n = (n + 1) / 2)
    hipLaunchKernelGGL(k_bcr_fwd, dim3(((n + 1) / 2 + 3) / 4), dim3(256), 0, st, a, lvl, n);
  hipLaunchKernelGGL(k_bcr_tail_solve, dim3(1), dim3(64 * TAIL_WAVES_S), 0, st, a, lt, P > 0 ? nt : 0);
  // wide backward levels, last to first
  for (int lvl = lt - 1; lvl >= 0; --lvl) {
    int nl = P;
    for (int v = 0; v < lvl; ++v) nl = (nl + 1) / 2;
    hipLaunchKernelGGL(k_bcr_bwd, dim3((nl / 2 + 3) / 4), dim3(256), 0, st, a, lvl, nl);
  }
}

void set_bcr_smem_limits() {
  hipFuncSetAttribute((const void*)k_bcr_border, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)border_smem(BT_MAXT0));
  set_bcr2_smem_limits();
}

}  // namespace ahlp
