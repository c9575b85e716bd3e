// Block cyclic reduction of the Schur complement (a6) for link pairs of 17 to
// 32 rows: the odd-even reduction of the one-tile kernels (k_bcr.hip) with
// every pair padded to 32 rows, i.e. a 2 x 2 block of 16x16 tiles.  The
// elimination of a pair o with active neighbours L and R is the same,
//   T'_oo = L_o L_o',  X_L = L_o^-1 T'_oL,  X_R = L_o^-1 T'_oR,  Z = L_o^-1 E'_o,
//   T'_LL -= X_L'X_L,  T'_RR -= X_R'X_R,  T'_RL = -X_R'X_L,
//   E'_L -= X_L'Z,  E'_R -= X_R'Z,
// with L_o a blocked Cholesky factor (two tile factorizations, one tile TRSM
// and update) and every product a sum of tile MFMA products.  Each level is
// one launch (the narrow ones too: a level costs a few microseconds either
// way), then the final pair, then the border as in the one-tile path.
//
// Storage (the BcrArgs arrays, sized for two tiles per pair side):
//   BD[j], BC[j], FLi[o], FXL[o], FXR[o]   2x2 tiles, tile (r, c) at c*2 + r
//   BEt[j], FGt[o]                         t0 x 2 tiles, tile (q, c) at c*t0 + q
// Pair vectors r, w, up: 32 values per pair.
#include "bcr_border.h"
#include "common.h"
#include "kernels.h"
#include "tile_chol.h"
#include "tile_ops.h"

namespace ahlp {

namespace {

constexpr int TP = 2;                  // tiles per pair side
constexpr int TB = 16 * TP;            // padded pair size
constexpr int BLK = TP * TP * 256;     // doubles per pair block
constexpr int MAXT0 = 4;               // border tiles (n0 <= 64)
constexpr int MID_WAVES = 16;          // waves of the final-pair and border solve kernel

// LDS tiles have leading dimension 17 (one pad value per column), so the
// accumulator-layout and B-operand accesses of a 16-lane row group fall in
// distinct banks.
constexpr int PLD = TS + 1;
constexpr int PT = 16 * PLD;           // values per LDS tile
constexpr int PBLK = TP * TP * PT;     // values per LDS pair block

// LDS of one eliminating wave (doubles).  During the factorization it holds
// X = L^-1, the working diagonal B, the inverted diagonal tiles and a scratch
// tile; once X is in registers (from which L^-1 also goes to global memory),
// the products X_L, X_R and Z' take the same space.  A workgroup's two regions
// take 68 KiB, so two workgroups share a CU.
constexpr int R_X = 0;                         // L^-1, TP x TP tiles
constexpr int R_B = PBLK;                      // working diagonal -> L
constexpr int R_LD = 2 * PBLK;                 // inverted diagonal tiles
constexpr int R_TMP = R_LD + TP * PT;
constexpr int R_XL = 0;                        // X_L (over X)
constexpr int R_XR = PBLK;                     // X_R (over B)
constexpr int R_GT = 2 * PBLK;                 // Z' (t0 x TP tiles, over Ld, tmp)
constexpr int R_SIZE = R_GT + MAXT0 * TP * PT;
static_assert(R_TMP + PT <= R_SIZE, "chol scratch outside the region");
static_assert(2 * R_SIZE * sizeof(double) <= 80 * 1024, "two workgroups per CU");

__device__ __forceinline__ long long et_off(long long j, int q, int cc, int t0) {
  return ((j * TP + cc) * t0 + q) * 256;
}
__device__ __forceinline__ int bt(int r, int cc) { return (cc * TP + r) * 256; }
__device__ __forceinline__ int pbt(int r, int cc) { return (cc * TP + r) * PT; }

// Working blocks from the assembled parts, one wave per tile: the diagonal
// (identity on the padding), the coupling T[j+1, j] and the border rows E_j'.
__global__ __launch_bounds__(256) void k_bcr2_init(BcrArgs c) {
  const int per = 2 * TP * TP + TP * c.t0;
  const long long wt = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wt >= (long long)c.P * per) return;
  const int j = (int)(wt / per), kind = (int)(wt % per), lj = c.l[j];
  if (kind < TP * TP) {
    const int r = kind % TP, cc = kind / TP;
    acc_store(c.BD + (long long)j * BLK + bt(r, cc),
              acc_load_exact(c.Td + c.tdoff[j] + 16 * r + 16LL * cc * lj, lj - 16 * r,
                             lj - 16 * cc, lj, r == cc));
  } else if (kind < 2 * TP * TP) {
    if (j + 1 < c.P) {
      const int t = kind - TP * TP, r = t % TP, cc = t / TP, ln = c.l[j + 1];
      acc_store(c.BC + (long long)j * BLK + bt(r, cc),
                acc_load_exact(c.To + c.tooff[j] + 16 * r + 16LL * cc * ln, ln - 16 * r,
                               lj - 16 * cc, ln, false));
    }
  } else {
    const int t = kind - 2 * TP * TP, q = t % c.t0, cc = t / c.t0;
    acc_store(c.BEt + et_off(j, q, cc, c.t0),
              acc_load_exact_t(c.E + c.eoff[j] + 16LL * q * lj + 16 * cc,
                               min(16, c.n0 - 16 * q), lj - 16 * cc, lj));
  }
}

// a tile as the B operand of X*Y (element (k, j) of the 16 x 4 slice s)
__device__ __forceinline__ Op op_load_b(const double* t) {
  const int lane = threadIdx.x & 63;
  const int idx = (lane & 15) * TS + (lane >> 4);
  Op o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[idx + 4 * s];
  return o;
}
// acc + alpha * (product of register operands)
__device__ __forceinline__ d4 mm(d4 acc, const Op& a, const Op& b, double alpha) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma(alpha * a.v[s], b.v[s], acc);
  return acc;
}

// Eliminate pair o: blocked Cholesky of its working diagonal, then
// X_L = L_o^-1 T'[o, L] (if needXL; T'[o, L] is BC[L]),
// X_R = L_o^-1 T'[R, o]' (if needXR; T'[R, o] is BC[o]) and
// Z' = E'_o' L_o^-T, all into the wave's LDS region R; L_o^-1 goes to fli
// (global, if not null) from registers.  Every global operand is loaded
// before the factorization, so the step waits on memory once.  Returns the
// pivots replaced.
__device__ int elim2(const BcrArgs& c, long long o, long long L, bool needXL, bool needXR,
                     double* R, double* fli) {
  const int t0 = c.t0;
  double* X = R + R_X;
  double* B = R + R_B;
  const double* D = c.BD + o * BLK;
  const double* CL = c.BC + L * BLK;
  const double* Co = c.BC + o * BLK;
  Op d00 = op_load(D + bt(0, 0)), d10 = op_load(D + bt(1, 0)), d11 = op_load(D + bt(1, 1));
  Op cl[TP][TP], co[TP][TP], et[TP][MAXT0];
#pragma unroll
  for (int q = 0; q < TP; ++q)
#pragma unroll
    for (int cc = 0; cc < TP; ++cc) {
      cl[q][cc] = needXL ? op_load_b(CL + bt(q, cc)) : Op{};
      co[cc][q] = needXR ? op_load(Co + bt(cc, q)) : Op{};
    }
#pragma unroll
  for (int p = 0; p < TP; ++p)
#pragma unroll
    for (int q = 0; q < MAXT0; ++q) et[p][q] = q < t0 ? op_load(c.BEt + et_off(o, q, p, t0)) : Op{};
  const double thr = c.thrT[o];
  op_store<PLD>(B + pbt(0, 0), d00);
  op_store<PLD>(B + pbt(1, 0), d10);
  op_store<PLD>(B + pbt(1, 1), d11);
  wave_order();
  const int cnt = wave_block_chol<PLD>(B, TP, X, R + R_LD, R + R_TMP, R + R_TMP, thr);
  wave_order();
  Op x[TP][TP];
#pragma unroll
  for (int r = 0; r < TP; ++r)
#pragma unroll
    for (int q = 0; q <= r; ++q) x[r][q] = op_load<PLD>(X + pbt(r, q));
  wave_order();   // X is read before the products overwrite it
  if (fli) {
#pragma unroll
    for (int r = 0; r < TP; ++r)
#pragma unroll
      for (int q = 0; q < TP; ++q) op_store(fli + bt(r, q), q <= r ? x[r][q] : Op{});
  }
#pragma unroll
  for (int r = 0; r < TP; ++r)
#pragma unroll
    for (int cc = 0; cc < TP; ++cc) {
      if (needXL) {
        d4 a = acc_zero();
#pragma unroll
        for (int q = 0; q <= r; ++q) a = mm(a, x[r][q], cl[q][cc], 1.0);
        acc_store<PLD>(R + R_XL + pbt(r, cc), a);
      }
      if (needXR) {
        d4 a = acc_zero();
#pragma unroll
        for (int q = 0; q <= r; ++q) a = mm(a, x[r][q], co[cc][q], 1.0);
        acc_store<PLD>(R + R_XR + pbt(r, cc), a);
      }
    }
  // Z'(q, cc) = sum_p E'(q, p) X(cc, p)'; X(cc, p) as the B operand of X*Y'
  // has the A-operand layout
#pragma unroll
  for (int cc = 0; cc < TP; ++cc)
#pragma unroll
    for (int q = 0; q < MAXT0; ++q)
      if (q < t0) {
        d4 a = acc_zero();
#pragma unroll
        for (int p = 0; p <= cc; ++p) a = mm(a, et[p][q], x[cc][p], 1.0);
        acc_store<PLD>(R + R_GT + (cc * t0 + q) * PT, a);
      }
  wave_order();
  return cnt;
}

// factor blocks X_L, X_R and Z' of pair o from the wave's LDS region
__device__ void store2(const BcrArgs& c, long long o, const double* R, bool hasL, bool hasR) {
  for (int t = 0; t < TP * TP; ++t) {
    if (hasL) tile_copy<TS, PLD>(c.FXL + o * BLK + t * 256, R + R_XL + t * PT);
    if (hasR) tile_copy<TS, PLD>(c.FXR + o * BLK + t * 256, R + R_XR + t * PT);
  }
  for (int t = 0; t < TP * c.t0; ++t)
    tile_copy<TS, PLD>(c.FGt + (o * TP * c.t0 + t) * 256, R + R_GT + t * PT);
}

// One level (n active pairs): a workgroup of two waves per even position k.
// Wave 0 eliminates the right neighbour o_r and stores its factor blocks,
// wave 1 eliminates the left neighbour o_l again (it is the right neighbour
// of k - 2, which stores it); then wave 0 updates the even pair's diagonal
// and new coupling, wave 1 its border rows, from both waves' products.
__global__ __launch_bounds__(128) void k_bcr2_level(BcrArgs c, int lvl, int n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int wave = threadIdx.x >> 6, k = 2 * blockIdx.x, t0 = c.t0;
  const long long s = 1LL << lvl, e = k * s;
  const bool hl = k >= 1, hr = k + 1 < n, hrr = k + 2 < n;
  int cnt = 0;
  // the even pair's own tiles, loaded before the elimination
  d4 dp[3], etp[TP][MAXT0];
  if (wave == 0) {
    double* D = c.BD + e * BLK;
    dp[0] = acc_load(D + bt(0, 0));
    dp[1] = acc_load(D + bt(1, 0));
    dp[2] = acc_load(D + bt(1, 1));
  } else {
#pragma unroll
    for (int cc = 0; cc < TP; ++cc)
#pragma unroll
      for (int q = 0; q < MAXT0; ++q)
        etp[cc][q] = q < t0 ? acc_load(c.BEt + et_off(e, q, cc, t0)) : acc_zero();
  }
  if (wave == 0 ? hr : hl) {
    double* R = lds + wave * R_SIZE;
    const long long o = wave == 0 ? (k + 1) * s : (k - 1) * s;
    const int cn = elim2(c, o, e, wave == 0, wave == 0 ? hrr : true, R,
                         wave == 0 ? c.FLi + o * BLK : nullptr);
    if (wave == 0) {
      cnt = cn;
      store2(c, o, R, true, hrr);
    }
  }
  __syncthreads();
  const double* Ro = lds;            // products of o_r
  const double* Rl = lds + R_SIZE;   // products of o_l
  if (wave == 0) {
    double* D = c.BD + e * BLK;
#pragma unroll
    for (int cc = 0; cc < TP; ++cc)
#pragma unroll
      for (int r = cc; r < TP; ++r) {
        d4 a = dp[cc + r];   // (0,0), (1,0), (1,1)
        if (hl)
          for (int p = 0; p < TP; ++p)
            a = mma_txy<PLD>(a, Rl + R_XR + pbt(p, r), Rl + R_XR + pbt(p, cc), -1.0);
        if (hr)
          for (int p = 0; p < TP; ++p)
            a = mma_txy<PLD>(a, Ro + R_XL + pbt(p, r), Ro + R_XL + pbt(p, cc), -1.0);
        acc_store(D + bt(r, cc), a);
      }
    if (hr && hrr)
      for (int cc = 0; cc < TP; ++cc)
        for (int r = 0; r < TP; ++r) {
          d4 a = acc_zero();
          for (int p = 0; p < TP; ++p)
            a = mma_txy<PLD>(a, Ro + R_XR + pbt(p, r), Ro + R_XL + pbt(p, cc), -1.0);
          acc_store(c.BC + e * BLK + bt(r, cc), a);
        }
  } else {
#pragma unroll
    for (int cc = 0; cc < TP; ++cc)
#pragma unroll
      for (int q = 0; q < MAXT0; ++q) {
        if (q >= t0) continue;
        double* Et = c.BEt + et_off(e, q, cc, t0);
        d4 a = etp[cc][q];
        if (hl)
          for (int p = 0; p < TP; ++p)
            a = mma_xy<PLD>(a, Rl + R_GT + (p * t0 + q) * PT, Rl + R_XR + pbt(p, cc), -1.0);
        if (hr)
          for (int p = 0; p < TP; ++p)
            a = mma_xy<PLD>(a, Ro + R_GT + (p * t0 + q) * PT, Ro + R_XL + pbt(p, cc), -1.0);
        acc_store(Et, a);
      }
  }
  if (threadIdx.x == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// the final pair (j = 0): L_0^-1 and Z_0'
__global__ __launch_bounds__(64) void k_bcr2_final(BcrArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* R = reinterpret_cast<double*>(smem_raw);
  const int cnt = elim2(c, 0, 0, false, false, R, c.FLi);
  store2(c, 0, R, false, false);
  if (threadIdx.x == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// ----------------------------------------------------------------- solve
// Forward: w_o = L_o^-1 r_o, r_e -= X_R(o_l)' w_{o_l} + X_L(o_r)' w_{o_r};
// backward: u_o = L_o^-T (w_o - X_L u_L - X_R u_R - Z_o u0).
struct Vec2 { double a[TB], b[TB], wl[TB], wr[TB], sc[16]; };

// element 16 h + lane % 16 of pair j's vector at level lvl (level 0: the
// exact right-hand side, zero on the padding)
__device__ __forceinline__ double rvec2(const BcrSolveArgs& A, int lvl, long long j, int h) {
  const int i = 16 * h + (threadIdx.x & 15);
  if (lvl == 0) return i < A.c.l[j] ? A.s[A.loff[j] + i] : 0.0;
  return A.r[j * TB + i];
}

// y = X v (lower: X is block lower triangular); v: TB values in LDS
__device__ __forceinline__ void blk_mv(const double* X, const double* v, bool lower, double* y) {
#pragma unroll
  for (int h = 0; h < TP; ++h) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < TP; ++q)
      if (!lower || q <= h) acc += op_mv(op_load(X + bt(h, q)), v + 16 * q);
    y[h] = acc;
  }
}
// y = X' v
__device__ __forceinline__ void blk_mtv(const double* X, const double* v, bool lower, double* sc,
                                        double* y) {
#pragma unroll
  for (int h = 0; h < TP; ++h) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < TP; ++q)
      if (!lower || q >= h) acc += op_mtv(op_load(X + bt(q, h)), v + 16 * q, sc);
    y[h] = acc;
  }
}
__device__ __forceinline__ void put2(double* dst, const double* y) {
  const int lane = threadIdx.x & 63;
  if (lane < 16) {
#pragma unroll
    for (int h = 0; h < TP; ++h) dst[16 * h + lane] = y[h];
  }
}
// border partial Z_o' w (w: TB values in LDS) into pb
__device__ __forceinline__ void border_partial(const BcrSolveArgs& A, long long o, const double* w) {
  const BcrArgs& c = A.c;
  const int lane = threadIdx.x & 63;
  for (int q = 0; q < c.t0; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int p = 0; p < TP; ++p) acc += op_mv(op_load(c.FGt + et_off(o, q, p, c.t0)), w + 16 * p);
    if (lane < 16) A.pb[(o * c.t0 + q) * 16 + lane] = acc;
  }
}

__device__ void fwd2_even(const BcrSolveArgs& A, int lvl, int n, int k, Vec2& V) {
  const BcrArgs& c = A.c;
  const int lane = threadIdx.x & 63;
  const long long s = 1LL << lvl, e = k * s, ol = (k - 1) * s, orr = (k + 1) * s;
  const bool hl = k >= 1, hr = k + 1 < n;
  double acc[TP], t[TP];
#pragma unroll
  for (int h = 0; h < TP; ++h) {
    acc[h] = rvec2(A, lvl, e, h);
    t[h] = hl ? rvec2(A, lvl, ol, h) : 0.0;
  }
  put2(V.a, t);
#pragma unroll
  for (int h = 0; h < TP; ++h) t[h] = hr ? rvec2(A, lvl, orr, h) : 0.0;
  put2(V.b, t);
  wave_order();
  if (hl) {
    blk_mv(c.FLi + ol * BLK, V.a, true, t);
    put2(V.wl, t);
  }
  if (hr) {
    blk_mv(c.FLi + orr * BLK, V.b, true, t);
    put2(V.wr, t);
  }
  wave_order();
  if (hl) {
    blk_mtv(c.FXR + ol * BLK, V.wl, false, V.sc, t);
#pragma unroll
    for (int h = 0; h < TP; ++h) acc[h] -= t[h];
  }
  if (hr) {
    blk_mtv(c.FXL + orr * BLK, V.wr, false, V.sc, t);
#pragma unroll
    for (int h = 0; h < TP; ++h) acc[h] -= t[h];
    if (lane < 16)
      for (int i = 0; i < TB; i += 16) A.w[orr * TB + i + lane] = V.wr[i + lane];
    border_partial(A, orr, V.wr);
  }
  if (lane < 16) {
#pragma unroll
    for (int h = 0; h < TP; ++h) A.r[e * TB + 16 * h + lane] = acc[h];
  }
  wave_order();
}

// u_o from w_o, the neighbours' u (L, R < 0: no such neighbour) and u0
__device__ void bwd2_pair(const BcrSolveArgs& A, long long o, long long L, long long R,
                          const double* u0, Vec2& V) {
  const BcrArgs& c = A.c;
  const int lane = threadIdx.x & 63;
  double v[TP], t[TP];
#pragma unroll
  for (int h = 0; h < TP; ++h) {
    v[h] = A.w[o * TB + 16 * h + (lane & 15)];
    t[h] = L >= 0 ? A.up[L * TB + 16 * h + (lane & 15)] : 0.0;
  }
  put2(V.a, t);
#pragma unroll
  for (int h = 0; h < TP; ++h) t[h] = R >= 0 ? A.up[R * TB + 16 * h + (lane & 15)] : 0.0;
  put2(V.b, t);
  wave_order();
  if (L >= 0) {
    blk_mv(c.FXL + o * BLK, V.a, false, t);
#pragma unroll
    for (int h = 0; h < TP; ++h) v[h] -= t[h];
  }
  if (R >= 0) {
    blk_mv(c.FXR + o * BLK, V.b, false, t);
#pragma unroll
    for (int h = 0; h < TP; ++h) v[h] -= t[h];
  }
#pragma unroll
  for (int h = 0; h < TP; ++h)
    for (int q = 0; q < c.t0; ++q) v[h] -= op_mtv(op_load(c.FGt + et_off(o, q, h, c.t0)), u0 + 16 * q, V.sc);
  put2(V.wl, v);
  wave_order();
  blk_mtv(c.FLi + o * BLK, V.wl, true, V.sc, t);
  if (lane < 16) {
    const int lo = c.l[o];
#pragma unroll
    for (int h = 0; h < TP; ++h) {
      A.up[o * TB + 16 * h + lane] = t[h];
      if (16 * h + lane < lo) A.u[A.loff[o] + 16 * h + lane] = t[h];
    }
  }
  wave_order();
}

__global__ __launch_bounds__(256) void k_bcr2_fwd(BcrSolveArgs A, int lvl, int n) {
  __shared__ Vec2 V[4];
  const int wave = threadIdx.x >> 6, w = blockIdx.x * 4 + wave;
  if (w >= (n + 1) / 2) return;
  fwd2_even(A, lvl, n, 2 * w, V[wave]);
}

__global__ __launch_bounds__(256) void k_bcr2_bwd(BcrSolveArgs A, int lvl, int n) {
  __shared__ Vec2 V[4];
  __shared__ double u0[16 * MAXT0];
  const int wave = threadIdx.x >> 6, w = blockIdx.x * 4 + wave;
  for (int i = threadIdx.x; i < 16 * A.c.t0; i += blockDim.x) u0[i] = A.u0p[i];
  __syncthreads();
  if (w >= n / 2) return;
  const int k = 2 * w + 1;
  const long long s = 1LL << lvl;
  bwd2_pair(A, k * s, (k - 1) * s, k + 1 < n ? (k + 1) * s : -1, u0, V[wave]);
}

// The final pair forward (w_0 = L_0^-1 r_0 and its border partial), the
// border solve, the final pair backward.  lvl: the level after the last
// reduction (where pair 0's right-hand side is).
__global__ __launch_bounds__(64 * MID_WAVES) void k_bcr2_mid(BcrSolveArgs A, int lvl) {
  const BcrArgs& c = A.c;
  __shared__ Vec2 V;
  __shared__ double part[64 * MID_WAVES];
  __shared__ double s0[16 * MAXT0], w0[16 * MAXT0], u0[16 * MAXT0];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (c.P >= 1 && wave == 0) {
    double t[TP];
#pragma unroll
    for (int h = 0; h < TP; ++h) t[h] = rvec2(A, lvl, 0, h);
    put2(V.a, t);
    wave_order();
    blk_mv(c.FLi, V.a, true, t);
    put2(V.wl, t);
    wave_order();
    if (lane < 16)
      for (int i = 0; i < TB; i += 16) A.w[i + lane] = V.wl[i + lane];
    border_partial(A, 0, V.wl);
  }
  __syncthreads();
  bcr_border_solve(A, A.c.FLbi, false, part, s0, w0, u0, V.sc);
  if (c.P >= 1 && wave == 0) bwd2_pair(A, 0, -1, -1, u0, V);
}

constexpr size_t LEVEL_SMEM = 2 * R_SIZE * sizeof(double);
constexpr size_t FINAL_SMEM = R_SIZE * sizeof(double);

}  // namespace

void launch_bcr2_reduce(hipStream_t st, const BcrArgs& c) {
  if (c.P <= 0) return;
  const long long tiles = (long long)c.P * (2 * TP * TP + TP * c.t0);
  hipLaunchKernelGGL(k_bcr2_init, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, c);
  int n = c.P, lvl = 0;
  for (; n > 1; ++lvl, n = (n + 1) / 2)
    hipLaunchKernelGGL(k_bcr2_level, dim3((n + 1) / 2), dim3(128), LEVEL_SMEM, st, c, lvl, n);
  hipLaunchKernelGGL(k_bcr2_final, dim3(1), dim3(64), FINAL_SMEM, st, c);
}

void launch_bcr2_solve(hipStream_t st, const BcrSolveArgs& a) {
  const int P = a.c.P;
  int n = P, lvl = 0;
  for (; n > 1; ++lvl, n = (n + 1) / 2)
    hipLaunchKernelGGL(k_bcr2_fwd, dim3(((n + 1) / 2 + 3) / 4), dim3(256), 0, st, a, lvl, n);
  hipLaunchKernelGGL(k_bcr2_mid, dim3(1), dim3(64 * MID_WAVES), 0, st, a, lvl);
  for (int lv = lvl - 1; lv >= 0; --lv) {
    int nl = P;
    for (int v = 0; v < lv; ++v) nl = (nl + 1) / 2;
    hipLaunchKernelGGL(k_bcr2_bwd, dim3((nl / 2 + 3) / 4), dim3(256), 0, st, a, lv, nl);
  }
}

void set_bcr2_smem_limits() {
  hipFuncSetAttribute((const void*)k_bcr2_level, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)LEVEL_SMEM);
  hipFuncSetAttribute((const void*)k_bcr2_final, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)FINAL_SMEM);
}

}  // namespace ahlp
