// Factorization kernels: D-scaling (a1), block SYRK (a2), link columns (a1),
// bordered block Cholesky = Cholesky of M_i and W_i = L_i^-1 B_i (a3, a4),
// Schur contributions W_i' W_i and their deterministic assembly (a5).
//
// Per block i the "bordered" matrix
//     [ M_i    B_i ]      M_i = A_i D_i A_i' (+ delta I),   B_i = [A_i D_i F_i' | C_i]
//     [ B_i'   *   ]
// is stored as lower tiles packed by tile columns (columns 0..mt-1 only): the
// first mt tile rows hold M_i, the next kt tile rows hold B_i'.  A left-looking
// Cholesky over the first mt columns turns them into L_i and W_i' = B_i' L_i^-T
// in place; this is the partial factorization of the bordered matrix that
// stops after the m_i pivots of the block (Sec. 3.2 discusses the same
// construction with an incomplete LU of [K_i L_i'; L_i 0]).
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "tile_chol.h"

namespace ahlp {

// ---------------------------------------------------------------- a1: D
// One workgroup per block (and one for x_0).  Fills the padded D =
// (z/x + q + rho)^-1 (q: the upper bounds' W/S, or none) and keeps a copy of x
// and z for the solve phase; flags non-positive or non-finite input.
__global__ void k_prep(const BlockInfo* __restrict__ blk, int N, int n0, long long x0off,
                       long long d0off, const double* __restrict__ x,
                       const double* __restrict__ z, const double* __restrict__ q, double rho,
                       double* __restrict__ Dp, double* __restrict__ xs, double* __restrict__ zs,
                       DevInfo* info) {
  int i = blockIdx.x;
  long long xoff, dpoff;
  int n, np;
  if (i < N) {
    xoff = blk[i].xoff; dpoff = blk[i].dpoff; n = blk[i].n; np = TS * blk[i].nt;
  } else {
    xoff = x0off; dpoff = d0off; n = n0; np = (n0 + TS - 1) / TS * TS;
  }
  int bad = 0;
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    double d = 0.0;
    if (c < n) {
      double xv = x[xoff + c], zv = z[xoff + c];
      xs[xoff + c] = xv;
      zs[xoff + c] = zv;
      if (!(xv > 0.0) || !(zv > 0.0) || !isfinite(xv) || !isfinite(zv)) bad = 1;
      d = q ? 1.0 / (zv / xv + q[xoff + c] + rho) : 1.0 / (zv / xv + rho);
    }
    Dp[dpoff + c] = d;
  }
  if (bad) atomicOr(&info->nonfinite, 1);
}

template <typename T>
__device__ __forceinline__ void tile_copy_t(T* __restrict__ dst, const T* __restrict__ src) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) dst[64 * s + lane] = src[64 * s + lane];
}

// ---------------------------------------------------------------- a2: SYRK
// One 64x64 lower macro tile of one block per workgroup (4 waves, each 32x32 =
// 2x2 MFMA tiles).  Per tile column K of A, the 4 row tiles and 4 column tiles
// are staged through LDS (double buffered), two tile columns ahead in
// registers; D scales the column tiles as they are staged (the B operand's
// product with D formed once per element instead of once per wave).  Work items are ordered so
// that consecutive items of one block land on the same XCD (its private L2
// then serves the repeated panel reads).
//
// The stage loads are 16-byte vector loads, the same number for every
// workgroup and every step (rows past the block and columns past its end are
// clamped to valid tiles and zeroed when the stage is written to LDS), so the
// compiler waits only for the stage due and never for the one behind it.
template <typename T> struct Bits;
template <> struct Bits<double> { typedef long long type; };
template <> struct Bits<float> { typedef int type; };
template <typename T>
__device__ __forceinline__ T keep_if(T v, typename Bits<T>::type m) {
  return __builtin_bit_cast(T, __builtin_bit_cast(typename Bits<T>::type, v) & m);
}

template <typename T>
__global__ __launch_bounds__(256) void k_syrk(const BlockInfo* __restrict__ blk,
                                              const int4* __restrict__ items, int nitems,
                                              const T* __restrict__ A,
                                              const double* __restrict__ Dp,
                                              T* __restrict__ LB, double delta) {
  typedef typename Bits<T>::type B;
  constexpr int E = 16 / sizeof(T);             // elements per 16-byte load
  constexpr int NJ = 8 * TE / (E * 256);        // loads per thread and stage
  typedef T V __attribute__((ext_vector_type(E)));
  int w = blockIdx.x;
  int per = gridDim.x / 8;
  int g = (w % 8) * per + (w / 8);
  if (g >= nitems) return;
  const int4 it = items[g];
  const BlockInfo b = blk[it.x];
  const int R0 = it.y * 4, C0 = it.z * 4;
  const bool diag = (it.y == it.z);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  // output tiles a wave computes: those stored, i.e. inside the block and on
  // or below the diagonal (a wave on the diagonal of a diagonal item skips
  // its upper tile (0, 1); waves past a ragged block's last tile row or
  // column skip theirs)
  const int I0 = R0 + 2 * wr, J0 = C0 + 2 * wc;
  bool use[2][2];
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
      use[tr][tc] = I0 + tr < b.mt && J0 + tc < b.mt && I0 + tr >= J0 + tc;
  const bool active = use[0][0] || use[0][1] || use[1][0] || use[1][1];

  typedef typename Acc<T>::type AT;
  AT acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = AT{0, 0, 0, 0};

  // load j of a thread: stage tile (f / 256) (0-3 row tiles, 4-7 column
  // tiles; a diagonal item loads its row tiles twice), elements f % 256 ..
  // + E - 1, f = (tid + 256 j) E.  Consecutive threads take consecutive 16
  // bytes, so a wave's load j fills 1 KiB of one tile: a direct-to-LDS load
  // writes it at the wave's base plus 16 bytes per lane, with no registers
  // in between.  Rows past the block read the last row tile again; the
  // products that would use them are skipped.
  const T* rbase[NJ];
  int ltile[NJ], lpe0[NJ];   // the wave's LDS destination of load j
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int f = (tid + 256 * j) * E, f0 = (64 * wave + 256 * j) * E;
    const int tl = f / TE;
    const int I = tl < 4 ? R0 + tl : C0 + tl - 4;
    rbase[j] = A + b.aoff + (long long)min(I, b.mt - 1) * b.nt * TE + f % TE;
    ltile[j] = f0 / TE;
    lpe0[j] = f0 % TE;
  }
  // two stage buffers as distinct arrays, so that loads into one do not make
  // the compiler wait before reads of the other
  __shared__ __align__(16) T sA0[8][TE];
  __shared__ __align__(16) T sA1[8][TE];
  __shared__ double sD0[TS], sD1[TS];
  const double* Dbase = Dp + b.dpoff + (tid & 15);
  double dreg = 0.0;
  auto stage = [&](auto bufc, int K) {   // stage K's tiles into buffer bufc
    constexpr int BUF = decltype(bufc)::value;
    const long long Kc = min(K, b.nt - 1);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      T* dst = BUF ? &sA1[ltile[j]][lpe0[j]] : &sA0[ltile[j]][lpe0[j]];
      __builtin_amdgcn_global_load_lds((const void*)(rbase[j] + Kc * TE),
                                       (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
    dreg = Dbase[Kc * TS];
  };
  auto step = [&](auto bufc, int K) {
    constexpr int BUF = decltype(bufc)::value;
    double* sD = BUF ? sD1 : sD0;
    if (tid < TS) sD[tid] = dreg;
    // every wave's direct-to-LDS loads of stage K complete before the barrier
    // (the barrier's own fence orders LDS and need not wait for them)
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    if (K + 1 < b.nt) stage(std::integral_constant<int, 1 - BUF>{}, K + 1);
    if (active && K < b.nt) {
      const T* ra0 = BUF ? sA1[2 * wr] : sA0[2 * wr];
      const T* ra1 = BUF ? sA1[2 * wr + 1] : sA0[2 * wr + 1];
      const T* cb0 = BUF ? sA1[4 + 2 * wc] : sA0[4 + 2 * wc];
      const T* cb1 = cb0 + TE;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        T a0 = ra0[64 * s + lane], a1 = ra1[64 * s + lane];
        T dd = (T)sD[4 * s + (lane >> 4)];
        T b0 = cb0[64 * s + lane] * dd, b1 = cb1[64 * s + lane] * dd;
        if (use[0][0]) acc[0][0] = mfma(a0, b0, acc[0][0]);
        if (use[0][1]) acc[0][1] = mfma(a0, b1, acc[0][1]);
        if (use[1][0]) acc[1][0] = mfma(a1, b0, acc[1][0]);
        if (use[1][1]) acc[1][1] = mfma(a1, b1, acc[1][1]);
      }
    }
  };
  stage(std::integral_constant<int, 0>{}, 0);
  for (int K = 0; K < b.nt; K += 2) {
    step(std::integral_constant<int, 0>{}, K);
    step(std::integral_constant<int, 1>{}, K + 1);
  }
  if (!active) return;
#pragma unroll
  for (int tr = 0; tr < 2; ++tr) {
#pragma unroll
    for (int tc = 0; tc < 2; ++tc) {
      const int I = I0 + tr, J = J0 + tc;
      if (!use[tr][tc]) continue;
      T* dst = LB + lb_tile(b, I, J);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = acc[tr][tc][r];
        const int i = acc_row<T>(lane, r), j = lane & 15;
        if (I == J && i == j) v = (TS * I + i < b.m) ? (T)(v + delta) : T(1);
        dst[acc_index<T>(lane, r)] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- a1: B_i'
// One workgroup per (block, tile row of the link columns).  Writes B_i' =
// [F_i D_i A_i' ; C_i'] into the bordered rows and F_i D_i F_i' (FP64) into the
// Schur-contribution tiles, F_i being block i's part of its two link pairs
// and of the global rows.  These rows are sparse (compressed rows, sorted
// columns), so the products are gathers rather than GEMMs.
// Tile row rr of block b's link columns, by 256 threads (t = 0..255).
template <typename T>
__device__ __forceinline__ void link_tile_row(const BlockInfo& b, int rr, int t, int nb,
                                              const double* __restrict__ A,
                                              const double* __restrict__ C,
                                              const int* __restrict__ lptr,
                                              const int* __restrict__ lcol,
                                              const double* __restrict__ lval,
                                              const double* __restrict__ Dp,
                                              T* __restrict__ LB, double* __restrict__ PQ) {
  const int r = b.mt + rr;
  const int ql = t & 15, al = t >> 4;
  const int q = TS * rr + ql;
  int qi;
  bool real;
  const int sec = link_section(b, q, &qi, nb, &real);
  const bool is_row = link_is_row(b, sec, qi);
  int p0 = 0, p1 = 0;
  if (real && is_row) {
    p0 = lptr[b.csr_off + q];
    p1 = lptr[b.csr_off + q + 1];
  }
  // LINK_CB column tiles at a time, their gathers independent so that they
  // are all in flight together; the sparse row is walked once per chunk
  constexpr int LINK_CB = 8;
  for (int c0 = 0; c0 < b.mt; c0 += LINK_CB) {
    double v[LINK_CB];
#pragma unroll
    for (int u = 0; u < LINK_CB; ++u) v[u] = 0.0;
    if (real && is_row) {
      for (int e = p0; e < p1; ++e) {
        const int j = lcol[e];
        const double coef = lval[e] * Dp[b.dpoff + j];
        const double* col = A + a_tile(b, 0, j >> 4) + (j & 15) * TS + al;
#pragma unroll
        for (int u = 0; u < LINK_CB; ++u) {
          const int c = c0 + u;
          if (c < b.mt && TS * c + al < b.m) v[u] += coef * col[(long long)c * b.nt * TE];
        }
      }
    } else if (real) {
      const int qc = qi - b.ng;   // column of C_i
      const double* col = C + c_tile(b, 0, qc >> 4) + (qc & 15) * TS + al;
#pragma unroll
      for (int u = 0; u < LINK_CB; ++u) {
        const int c = c0 + u;
        if (c < b.mt && TS * c + al < b.m) v[u] = col[(long long)c * b.kc0 * TE];
      }
    }
#pragma unroll
    for (int u = 0; u < LINK_CB; ++u)
      if (c0 + u < b.mt) LB[lb_tile(b, r, c0 + u) + t] = (T)v[u];
  }
  // F D F' for tiles (rr, cc), cc <= rr
  for (int cc = 0; cc <= rr; ++cc) {
    const int q2 = TS * cc + al;
    int qi2;
    bool real2;
    const int sec2 = link_section(b, q2, &qi2, nb, &real2);
    double v = 0.0;
    if (real && real2 && is_row && link_is_row(b, sec2, qi2)) {
      int e1 = p0, e2 = lptr[b.csr_off + q2];
      const int e2end = lptr[b.csr_off + q2 + 1];
      while (e1 < p1 && e2 < e2end) {
        const int j1 = lcol[e1], j2 = lcol[e2];
        if (j1 == j2) {
          v += lval[e1] * Dp[b.dpoff + j1] * lval[e2];
          ++e1; ++e2;
        } else if (j1 < j2) {
          ++e1;
        } else {
          ++e2;
        }
      }
    }
    PQ[pq_tile(b, rr, cc) + t] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_link(const BlockInfo* __restrict__ blk,
                                              const int2* __restrict__ items, int nb,
                                              const double* __restrict__ A,
                                              const double* __restrict__ C,
                                              const int* __restrict__ lptr,
                                              const int* __restrict__ lcol,
                                              const double* __restrict__ lval,
                                              const double* __restrict__ Dp,
                                              T* __restrict__ LB, double* __restrict__ PQ) {
  const int2 it = items[blockIdx.x];
  link_tile_row<T>(blk[it.x], it.y, threadIdx.x, nb, A, C, lptr, lcol, lval, Dp, LB, PQ);
}

// ---------------------------------------------------------------- a3 + a4
// One workgroup per block: left-looking blocked Cholesky over the mt tile
// columns of the bordered matrix.  Column panel p is first updated with the
// finished columns (MFMA, A operand = L(r,q), B operand = L(p,q)'), its
// diagonal tile is factored and inverted by one wave, and the tiles below are
// multiplied by the inverse's transpose (MFMA).  The inverted diagonal tiles
// are kept for the solve phase.
template <typename T>
__global__ __launch_bounds__(256) void k_block_factor(const BlockInfo* __restrict__ blk,
                                                      const int* __restrict__ order,
                                                      T* __restrict__ LB, T* __restrict__ LINV,
                                                      DevInfo* info) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BlockInfo b = blk[order[blockIdx.x]];
  // LDS tiles with leading dimension 17 (see the panel kernel)
  constexpr int LD = TS + 1, TEP = TS * LD, AST = sizeof(T) == 8 ? 4 : 1;
  T* panel = reinterpret_cast<T*>(smem_raw);
  T* linv = panel + (size_t)b.rt * TEP;
  __shared__ double s_max[4];
  __shared__ T xbuf[48];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  typedef typename Acc<T>::type AT;
  const int wb = (lane & 15) * LD + (sizeof(T) == 8 ? (lane >> 4) : 4 * (lane >> 4));
  const int rb = lane + (lane >> 4), tb = tid + (tid >> 4);

  // pivot threshold from the largest real diagonal entry of M_i
  double md = 0.0;
  for (int idx = tid; idx < b.m; idx += blockDim.x) {
    const int p = idx >> 4, i = idx & 15;
    md = fmax(md, (double)LB[lb_tile(b, p, p) + i * 17]);
  }
  for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off));
  if (lane == 0) s_max[wave] = md;
  __syncthreads();
  const double thr = PIVOT_REL * fmax(fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3])), 0.0);
  int cnt = 0;

  for (int p = 0; p < b.mt; ++p) {
    for (int r = p + wave; r < b.rt; r += 4) {
      AT acc;
      const T* src = LB + lb_tile(b, r, p);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = src[acc_index<T>(lane, k)];
      for (int q = 0; q < p; ++q) {
        const T* X = LB + lb_tile(b, r, q);
        const T* Y = LB + lb_tile(b, p, q);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = mfma(-X[64 * s + lane], Y[64 * s + lane], acc);
      }
      T* dst = panel + (size_t)(r - p) * TEP;
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[wb + AST * k] = acc[k];
    }
    __syncthreads();
    if (wave == 0) cnt += wave_chol_tile<T, LD>(panel, panel, linv, thr, xbuf);
    __syncthreads();
    LB[lb_tile(b, p, p) + tid] = panel[tb];
    LINV[b.linvoff + (long long)p * TE + tid] = linv[tb];
    for (int r = p + 1 + wave; r < b.rt; r += 4) {
      AT acc = AT{0, 0, 0, 0};
      const T* X = panel + (size_t)(r - p) * TEP;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma(X[rb + 68 * s], linv[rb + 68 * s], acc);
      T* dst = LB + lb_tile(b, r, p);
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[acc_index<T>(lane, k)] = acc[k];
    }
    __syncthreads();
  }
  if (tid == 0 && cnt) atomicAdd(&info->pivots, cnt);
}

// Schur contribution of block i: PQ = F D F' - X X' with X = W_i' (the
// bordered rows of the factor), in FP64 whatever the factor precision.  The
// workgroup's nw waves take the tile rows rr = w, w + nw, ...; row rr's tiles
// (rr, cc), cc <= rr, go in groups of SC_G sharing the loads of X(rr, q), and
// the tiles of step q + 1 are requested before the MFMAs of step q.
template <typename T>
__device__ __forceinline__ void schur_rows(const BlockInfo& b, const T* __restrict__ LB,
                                           double* __restrict__ PQ, int w, int lane, int nw = 4) {
  constexpr int SC_G = 4;
  for (int rr = w; rr < b.kt; rr += nw) {
    for (int cg = 0; cg <= rr; cg += SC_G) {
      const int ng = min(SC_G, rr + 1 - cg);
      d4 acc[SC_G];
#pragma unroll
      for (int u = 0; u < SC_G; ++u) {
        acc[u] = d4{0.0, 0.0, 0.0, 0.0};
        if (u < ng) {
          const double* dst = PQ + pq_tile(b, rr, cg + u);
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[u][k] = dst[acc_index<double>(lane, k)];
        }
      }
      T xc[4], yc[SC_G][4], xn[4], yn[SC_G][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) xc[s] = LB[lb_tile(b, b.mt + rr, 0) + 64 * s + lane];
#pragma unroll
      for (int u = 0; u < SC_G; ++u)
        if (u < ng) {
#pragma unroll
          for (int s = 0; s < 4; ++s) yc[u][s] = LB[lb_tile(b, b.mt + cg + u, 0) + 64 * s + lane];
        }
      for (int q = 0; q < b.mt; ++q) {
        const bool more = q + 1 < b.mt;
        if (more) {
#pragma unroll
          for (int s = 0; s < 4; ++s) xn[s] = LB[lb_tile(b, b.mt + rr, q + 1) + 64 * s + lane];
#pragma unroll
          for (int u = 0; u < SC_G; ++u)
            if (u < ng) {
#pragma unroll
              for (int s = 0; s < 4; ++s) yn[u][s] = LB[lb_tile(b, b.mt + cg + u, q + 1) + 64 * s + lane];
            }
        }
#pragma unroll
        for (int u = 0; u < SC_G; ++u)
          if (u < ng) {
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[u] = mfma(-(double)xc[s], (double)yc[u][s], acc[u]);
          }
        if (more) {
#pragma unroll
          for (int s = 0; s < 4; ++s) xc[s] = xn[s];
#pragma unroll
          for (int u = 0; u < SC_G; ++u)
#pragma unroll
            for (int s = 0; s < 4; ++s) yc[u][s] = yn[u][s];
        }
      }
#pragma unroll
      for (int u = 0; u < SC_G; ++u)
        if (u < ng) {
          double* dst = PQ + pq_tile(b, rr, cg + u);
#pragma unroll
          for (int k = 0; k < 4; ++k) dst[acc_index<double>(lane, k)] = acc[u][k];
        }
    }
  }
}


// Panel form of the same factorization for bordered blocks of at most
// BF_RMAX*4 tile rows: left-looking by panels of BF_PW tile columns held in
// registers (4 waves, panel rows dealt round-robin, at most BF_RMAX per wave).
// The update of a panel by each earlier tile column k reads L(r, k) for the
// wave's rows and L(c, k) for the panel columns, all issued together.  The panel is then factored
// column by column: Cholesky of the diagonal tile (its owner wave), the rows
// below times L_cc^-T (through a per-wave LDS conversion to operand layout),
// and the next panel column updated from an LDS copy of the new column.
// Two workgroups share a CU, so one block's tile Cholesky overlaps the
// other's MFMA work.  The kernel ends with the block's Schur contribution
// (schur_rows), so no separate a5 product pass is needed on this path.
// BF_RMAX is a template parameter: 5 (blocks of up to 20 tile rows) or 6 (up
// to 24, where the sixth row's accumulators fill the 256 VGPRs); a launch takes
// the smaller that fits its widest block.
constexpr int BF_PW = 2, BF_RMAX_MAX = 6;
static_assert(BF_PW == 2, "the pipelined panel update takes its steps in pairs");
// The panel kernel's LDS tiles are column-major with leading dimension 17:
// the accumulator layout writes a tile by columns across the lanes, which
// with 16 would put the 16 lanes of a row group in the same bank; with 17
// they fall in distinct banks, and the operand-layout reads stay contiguous.
// Per lane, the padded positions are a base plus a constant: accumulator
// element r of a double tile at wb + 4 r (float: wb + r), operand element s
// at rb + 68 s, with the bases computed once.
template <int BF_RMAX> struct BfLd { static constexpr int LD = TS + 1; };
template <int LD>
__device__ __forceinline__ int pidx(int e) { return LD == TS ? e : e + (e >> 4); }   // col 16 + row -> col LD + row
template <typename T>
struct BfOp { T v[4]; };
template <typename T>
__device__ __forceinline__ BfOp<T> bf_ld(const T* __restrict__ t) {
  const int lane = threadIdx.x & 63;
  BfOp<T> o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[64 * s + lane];
  return o;
}
// the same from an LDS tile of leading dimension LD
template <typename T, int LD>
__device__ __forceinline__ BfOp<T> bf_ld_p(const T* __restrict__ t) {
  const int lane = threadIdx.x & 63;
  BfOp<T> o;
#pragma unroll
  for (int s = 0; s < 4; ++s) o.v[s] = t[pidx<LD>(64 * s + lane)];
  return o;
}
// LDS tile of leading dimension LD to a plain tile in global memory
template <typename T, int LD>
__device__ __forceinline__ void tile_copy_p(T* __restrict__ dst, const T* __restrict__ src) {
  const int lane = threadIdx.x & 63;
  T v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = src[pidx<LD>(64 * s + lane)];
#pragma unroll
  for (int s = 0; s < 4; ++s) dst[64 * s + lane] = v[s];
}

// Synchronization of the panel factor's four waves in the standalone kernel:
// a workgroup barrier, and every panel's inputs are there from the start.
struct WgSync {
  static constexpr bool kPrefetch = true;
  __device__ __forceinline__ void sync() { __syncthreads(); }
  __device__ __forceinline__ bool wait_panel(int) { return true; }
};

// Largest real diagonal entry of block b's M_i (threads 0..255, all of which
// call it; s_max: 4 doubles of LDS).
template <typename T, int NW, class Sync>
__device__ __forceinline__ double block_diag_max(const BlockInfo& b, const T* __restrict__ LB,
                                                 double* s_max, Sync& sy) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double md = 0.0;
  for (int idx = tid; idx < b.m; idx += 64 * NW) {
    const int p = idx >> 4, i = idx & 15;
    md = fmax(md, (double)LB[lb_tile(b, p, p) + i * 17]);
  }
  for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off));
  if (lane == 0) s_max[w] = md;
  sy.sync();
  double r = s_max[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) r = fmax(r, s_max[k]);
  return r;
}

// The panel factorization of one bordered block by NW waves, with pivot
// threshold thr; smem_raw is its dynamic LDS.  Sync provides the barrier of
// the waves and the wait for the inputs of panel c0 (returns false when the
// wait was abandoned, and the factorization stops).
//
// The block's Schur contribution PQ - W_i'W_i (W_i' = the bordered rows) is a
// sum over the tile columns q, in FP64 in both precisions.  When its
// kt(kt+1)/2 FP64 tiles fit in the sch_cap LDS tiles after the per-wave
// ones, the waves that never factor a
// diagonal tile (w >= BF_PW) add column q's terms while a later column's
// diagonal tile is being factored, from the panel column buffer that still
// holds column q: the same products in the same order as schur_rows at the
// end, which otherwise re-reads every W tile from memory.
template <typename T, int BF_RMAX, int NW, class Sync>
__device__ __forceinline__ void panel_factor(const BlockInfo& b, T* __restrict__ LB,
                                             T* __restrict__ LINV, double* __restrict__ PQ,
                                             DevInfo* info, unsigned char* smem_raw, double thr,
                                             Sync& sy, int sch_cap = 0) {
  constexpr int LD = BfLd<BF_RMAX>::LD, TEP = TS * LD;
  constexpr int AST = sizeof(T) == 8 ? 4 : 1;   // accumulator element stride in a padded tile
  const int mt = b.mt, rt = b.rt;
  // FP64 keeps every panel tile transposed in its accumulators (X' instead of
  // X): in the FP64 accumulator layout, register s of X' is exactly the B
  // operand of K-slice s, so the solve with L_cc^-1 and the panel's own
  // updates take X' straight from registers.  (The FP32 layout does not line
  // up this way; it converts through LDS.)
  constexpr bool TR = sizeof(T) == 8;
  T* colbuf = reinterpret_cast<T*>(smem_raw);          // rt tiles: the panel column just factored
  T* li = colbuf + (size_t)rt * TEP;                    // L_cc^-1
  T* dt = li + TEP;                                     // diagonal tile / its factor
  T* scr = dt + TEP;                                    // NW tiles: per-wave conversion
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: row and address arithmetic stays scalar
  typedef typename Acc<T>::type AT;
  int cnt = 0;
  T* myscr = scr + w * TEP;
  // padded positions of this lane's accumulator elements (wb + AST r) and
  // operand elements (rb + 68 s)
  const int wb = (lane & 15) * LD + (sizeof(T) == 8 ? (lane >> 4) : 4 * (lane >> 4));
  const int rb = lane + (lane >> 4);
  auto st_acc = [&](T* t, const AT& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) t[wb + AST * k] = a[k];
  };
  auto ld_op = [&](const T* t) {
    BfOp<T> o;
#pragma unroll
    for (int s = 0; s < 4; ++s) o.v[s] = t[rb + 68 * s];
    return o;
  };
  // Schur contribution in the factorization's gaps (FP64 accumulators in
  // LDS): tile u of the kt(kt+1)/2 lower tiles (row-major over (rr, cc), cc <= rr) belongs to
  // worker wave BF_PW + u % (NW - BF_PW), which alone reads and writes it
  const int kt = b.kt, nst = kt * (kt + 1) / 2;
  const bool sgap = NW > BF_PW && nst > 0 && nst <= sch_cap;
  double* sacc = reinterpret_cast<double*>(scr + NW * TEP);   // nst tiles, accumulator layout
  const int sb = (lane & 15) * LD + (lane >> 4);   // FP64 accumulator element k at sb + 4 k
  int qpend = -1, qc0 = 0;   // column whose terms are pending, and its panel's first column
  auto schur_col = [&](int c0q) {   // the pending column, factored in the panel at c0q
    int rr = 0, cc = 0;
    for (int u = 0; u < nst; ++u) {
      if (u % (NW - BF_PW) == w - BF_PW) {
        const BfOp<T> x = ld_op(colbuf + (size_t)(mt + rr - c0q) * TEP);
        const BfOp<T> y = ld_op(colbuf + (size_t)(mt + cc - c0q) * TEP);
        double* t = sacc + (size_t)u * TEP;
        d4 a;
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = t[sb + 4 * k];
#pragma unroll
        for (int s = 0; s < 4; ++s) a = mfma(-(double)x.v[s], (double)y.v[s], a);
#pragma unroll
        for (int k = 0; k < 4; ++k) t[sb + 4 * k] = a[k];
      }
      if (++cc > rr) { ++rr; cc = 0; }
    }
  };
  if (sgap && w >= BF_PW) {
    int rr = 0, cc = 0;
    for (int u = 0; u < nst; ++u) {
      if (u % (NW - BF_PW) == w - BF_PW) {
        const double* src = PQ + pq_tile(b, rr, cc);
#pragma unroll
        for (int k = 0; k < 4; ++k) sacc[(size_t)u * TEP + sb + 4 * k] = src[acc_index<double>(lane, k)];
      }
      if (++cc > rr) { ++rr; cc = 0; }
    }
  }

  // Prefetch into L2 (standalone kernel): the next panel's input tiles (the
  // SYRK's and the link gather's, written long before and mostly out of L2
  // by now) are requested while the current panel's second diagonal tile is
  // factored.  One lane touches each 128-byte line, with a direct-to-LDS
  // load into a scratch area nobody reads, so no registers are held.  (A
  // wave's next LDS write waits for its direct-to-LDS loads, so the
  // factoring wave issues none.)
  constexpr int LPT = TE * (int)sizeof(T) / 128;   // lines per tile
  constexpr int TPI = 64 / LPT;                     // tiles per prefetch instruction
  __shared__ __align__(16) unsigned char pf_sink[256];
  auto touch = [&](bool valid, const T* tile) {
    if (valid)
      __builtin_amdgcn_global_load_lds(
          (const void*)(reinterpret_cast<const char*>(tile) + (lane % LPT) * 128),
          (__attribute__((address_space(3))) void*)pf_sink, 4, 0, 0);
  };
  // tiles of panel n0 (column n0 + j, rows n0 + j .. rt - 1), dealt to the
  // NW - 1 waves other than skip
  auto prefetch_panel = [&](int n0, int skip) {
    const int npw = min(BF_PW, mt - n0);
    const int me = w < skip ? w : w - 1;
    const int n1 = rt - n0, ntile = n1 + (npw > 1 ? n1 - 1 : 0);
    for (int u0 = me * TPI; u0 < ntile; u0 += (NW - 1) * TPI) {
      const int u = u0 + lane / LPT;
      const int j = u < n1 ? 0 : 1, r = u < n1 ? n0 + u : n0 + 1 + (u - n1);
      touch(u < ntile, LB + lb_tile(b, min(r, rt - 1), n0 + j));
    }
  };
  for (int c0 = 0; c0 < mt; c0 += BF_PW) {
    const int pw = min(BF_PW, mt - c0);
    if (!sy.wait_panel(c0)) return;
    // rows r = c0 + w + NW t of this panel owned by the wave
    AT acc[BF_RMAX][BF_PW];
#pragma unroll
    for (int t = 0; t < BF_RMAX; ++t) {
      const int r = c0 + w + NW * t;
#pragma unroll
      for (int j = 0; j < BF_PW; ++j) {
        acc[t][j] = AT{0, 0, 0, 0};
        if (r < rt && j < pw && r >= c0 + j) {
          const T* src = LB + lb_tile(b, r, c0 + j);
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[t][j][k] = src[TR ? 64 * k + lane : acc_index<T>(lane, k)];
        }
      }
    }
    // left-looking update with the tile columns before the panel
    if constexpr (BF_RMAX <= 5 && sizeof(T) == 4) {
      // FP32, software-pipelined: step k + 1's tiles are requested while step k's
      // products run.  A row's registers take its next tile as soon as the
      // row's products have been issued; the two panel-column tiles, which
      // every row needs first, are double-buffered.  Every load is
      // unconditional, so that the compiler waits for exactly the tiles a
      // product needs: a wave with fewer than BF_RMAX rows in the panel loads
      // the panel's first tile row (already in its cache) for the others, and
      // the last step requests its own tiles again.  (In FP64, where each
      // product takes twice as long, the same loop measured no faster:
      // the two blocks sharing the CU keep the matrix pipe busy while one
      // waits for its tiles.)
      int nrow = rt - c0 - w;
      nrow = nrow > 0 ? min(BF_RMAX, (nrow + NW - 1) / NW) : 0;
      BfOp<T> Ac[BF_RMAX], B0[BF_PW], B1[BF_PW];
      auto ld_b = [&](BfOp<T>* Bc, int k) {
#pragma unroll
        for (int j = 0; j < BF_PW; ++j) Bc[j] = bf_ld<T>(LB + lb_tile(b, min(c0 + j, rt - 1), k));
      };
      auto ld_a = [&](int t, int k) {
        Ac[t] = bf_ld<T>(LB + lb_tile(b, t < nrow ? c0 + w + NW * t : c0, k));
      };
      // the row's products
      auto row_mm = [&](int t, const BfOp<T>* Bc) {
        const int r = c0 + w + NW * t;
        if (t < nrow) {
#pragma unroll
          for (int j = 0; j < BF_PW; ++j)
            if (j < pw && r >= c0 + j)
#pragma unroll
              for (int s = 0; s < 4; ++s) acc[t][j] = mfma(-Ac[t].v[s], Bc[j].v[s], acc[t][j]);
        }
      };
      // the order of issue is fixed (no scheduling across these points)
      auto fence = [] { __builtin_amdgcn_sched_barrier(0); };
      // (issued in the first panel too, where nothing uses them: loads under
      // a branch would make the compiler wait for every earlier tile)
      fence();
      ld_b(B0, 0);
#pragma unroll
      for (int t = 0; t < BF_RMAX; ++t) {
        fence();
        ld_a(t, 0);
      }
      fence();
      for (int k = 0; k < c0; k += BF_PW) {   // c0 is a multiple of BF_PW = 2
        fence();
        ld_b(B1, k + 1);
#pragma unroll
        for (int t = 0; t < BF_RMAX; ++t) {
          fence();
          row_mm(t, B0);
          fence();
          ld_a(t, k + 1);
        }
        const int k2 = min(k + 2, c0 - 1);
        fence();
        ld_b(B0, k2);
#pragma unroll
        for (int t = 0; t < BF_RMAX; ++t) {
          fence();
          row_mm(t, B1);
          fence();
          ld_a(t, k2);
        }
        fence();
      }
    } else {
      // all loads of a step issued together
      for (int k = 0; k < c0; ++k) {
        BfOp<T> Ac[BF_RMAX], Bc[BF_PW];
#pragma unroll
        for (int t = 0; t < BF_RMAX; ++t) {
          const int r = c0 + w + NW * t;
          if (r < rt) Ac[t] = bf_ld<T>(LB + lb_tile(b, r, k));
        }
#pragma unroll
        for (int j = 0; j < BF_PW; ++j)
          if (j < pw) Bc[j] = bf_ld<T>(LB + lb_tile(b, c0 + j, k));
#pragma unroll
        for (int t = 0; t < BF_RMAX; ++t) {
          const int r = c0 + w + NW * t;
#pragma unroll
          for (int j = 0; j < BF_PW; ++j)
            if (r < rt && j < pw && r >= c0 + j)
#pragma unroll
              for (int s = 0; s < 4; ++s)
                acc[t][j] = TR ? mfma(-Bc[j].v[s], Ac[t].v[s], acc[t][j])
                               : mfma(-Ac[t].v[s], Bc[j].v[s], acc[t][j]);
        }
      }
    }
    // Every input and update load of the panel has been consumed.  Saying so
    // once here keeps the compiler's conservative wait for them (it cannot
    // tell a zero-trip update loop from a full one) out of the solves below,
    // where the outstanding memory operations are the previous rows' stores.
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    // factor the panel column by column
#pragma unroll
    for (int j = 0; j < BF_PW; ++j) {
      if (j >= pw) break;
      const int c = c0 + j;
      const int ow = (c - c0) % NW, ot = (c - c0) / NW;
      // the previous column's Schur terms while wave ow factors this one
      if (sgap && w >= BF_PW && qpend >= 0) schur_col(qc0);
      if (Sync::kPrefetch && j == BF_PW - 1 && c0 + BF_PW < mt && w != ow)
        prefetch_panel(c0 + BF_PW, ow);
      if (w == ow) {
#pragma unroll
        for (int t = 0; t < BF_RMAX; ++t)
          if (t == ot) {
            st_acc(dt, acc[t][j]);
          }
        wave_order();
        cnt += wave_chol_tile<T, LD>(dt, dt, li, thr, nullptr);
      }
      sy.sync();
      // rows below: L(r, c) = acc(r, c) L_cc^-T
      const BfOp<T> lio = ld_op(li);
#pragma unroll
      for (int t = 0; t < BF_RMAX; ++t) {
        const int r = c0 + w + NW * t;
        if (r < rt && r > c) {
          T* dst = LB + lb_tile(b, r, c);
          T* cb = colbuf + (size_t)(r - c0) * TEP;
          AT l = AT{0, 0, 0, 0};
          if constexpr (TR) {
            // L(r, c)' = L_cc^-1 X' with X' in the accumulator registers,
            // whose element s is the B operand of K-slice s; the result is
            // again L(r, c)' in accumulator layout (kept for the updates below)
#pragma unroll
            for (int s = 0; s < 4; ++s) l = mfma(lio.v[s], acc[t][j][s], l);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              dst[64 * k + lane] = l[k];
              cb[rb + 68 * k] = l[k];
            }
            acc[t][j] = l;
          } else {
            st_acc(myscr, acc[t][j]);
            wave_order();
            const BfOp<T> x = ld_op(myscr);
#pragma unroll
            for (int s = 0; s < 4; ++s) l = mfma(x.v[s], lio.v[s], l);
            wave_order();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              dst[acc_index<T>(lane, k)] = l[k];
              cb[wb + AST * k] = l[k];
            }
          }
        }
      }
      // the diagonal tile's factor and inverse, needed only after the kernel,
      // go out now, off the chain (dt and li stay untouched until the next
      // barrier)
      if (w == ow) {
        tile_copy_p<T, LD>(LB + lb_tile(b, c, c), dt);
        tile_copy_p<T, LD>(LINV + b.linvoff + (long long)c * TE, li);
      }
      sy.sync();
      qpend = c;
      qc0 = c0;
      // the panel's later columns: acc(r, c') -= L(r, c) L(c', c)'
#pragma unroll
      for (int j2 = 0; j2 < BF_PW; ++j2) {
        if (j2 <= j || j2 >= pw) continue;
        const int c2 = c0 + j2;
        const BfOp<T> y = ld_op(colbuf + (size_t)(c2 - c0) * TEP);
#pragma unroll
        for (int t = 0; t < BF_RMAX; ++t) {
          const int r = c0 + w + NW * t;
          if (r < rt && r >= c2) {
            if constexpr (TR) {
              // X' -= L(c', c) L(r, c)': A operand from LDS, B operand the
              // row's own L(r, c)' registers
#pragma unroll
              for (int s = 0; s < 4; ++s) acc[t][j2] = mfma(-y.v[s], acc[t][j][s], acc[t][j2]);
            } else {
              const BfOp<T> x = ld_op(colbuf + (size_t)(r - c0) * TEP);
#pragma unroll
              for (int s = 0; s < 4; ++s) acc[t][j2] = mfma(-x.v[s], y.v[s], acc[t][j2]);
            }
          }
        }
      }
      sy.sync();
    }
  }
  if (sgap) {
    // the last column's terms, then the worker waves' tiles to PQ
    if (w >= BF_PW) {
      if (qpend >= 0) schur_col(qc0);
      int rr = 0, cc = 0;
      for (int u = 0; u < nst; ++u) {
        if (u % (NW - BF_PW) == w - BF_PW) {
          double* dst = PQ + pq_tile(b, rr, cc);
#pragma unroll
          for (int k = 0; k < 4; ++k) dst[acc_index<double>(lane, k)] = sacc[(size_t)u * TEP + sb + 4 * k];
        }
        if (++cc > rr) { ++rr; cc = 0; }
      }
    }
  } else {
    // the block's Schur contribution while its W' tiles are still in L2 (the
    // loop's last barrier has made every wave's stores visible)
    schur_rows<T>(b, LB, PQ, w, lane, NW);
  }
  // each wave counts the pivots of the diagonal tiles it factored
  if (lane == 0 && cnt) atomicAdd(&info->pivots, cnt);
}

// Standalone panel kernel: NW waves per block (4: two workgroups per CU, for
// bordered blocks of up to 4 BF_RMAX tile rows; 8: one per CU, up to
// 8 BF_RMAX).
template <typename T, int BF_RMAX, int NW>
__global__ __launch_bounds__(64 * NW, 8 / NW) void k_block_factor_panel(
    const BlockInfo* __restrict__ blk, const int* __restrict__ order, T* __restrict__ LB,
    T* __restrict__ LINV, double* __restrict__ PQ, DevInfo* info, int sch_cap) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double s_max[NW];
  const BlockInfo b = blk[order[blockIdx.x]];
  WgSync sy;
  const double thr = PIVOT_REL * fmax(block_diag_max<T, NW>(b, LB, s_max, sy), 0.0);
  panel_factor<T, BF_RMAX, NW>(b, LB, LINV, PQ, info, smem_raw, thr, sy, sch_cap);
}

// ------------------------------------------------- a1-a5 in one launch
// One persistent launch for the blocks of the panel bucket: a workgroup of
// eight waves per CU.  Waves 4-7 (the SYRK team) take blocks from a queue in
// the bucket's order (largest first) and form, per block, the link columns
// (link_tile_row), then the diagonal 32x32 wave tiles of M_i, then the
// off-diagonal ones column by column; waves 0-3 (the factor team) run the
// panel factorization of the block the SYRK team started, panel by panel as
// soon as the tile columns it needs are complete, while the SYRK team goes on
// with the next block.  So a block's latency-bound factorization chain runs
// beside the next block's MFMA-bound SYRK on the same CU.  Every value is
// computed by the same arithmetic in the same order as in the separate
// kernels (k_link, k_syrk, k_block_factor_panel), so the factors are
// bitwise the same.
//
// The two teams meet through LDS only: a ring of two block slots, each with
// its block, a sequence number and completion counters (link rows, diagonal
// wave tiles, off-diagonal wave tiles per tile-column pair) and the largest
// diagonal entry (for the pivot threshold); a producer stores its tiles,
// fences at workgroup scope and bumps a counter; a consumer waits for the
// count and fences.  The factor team's own barrier is an LDS counter (a
// workgroup barrier would also wait for the SYRK team).  Every wait is
// bounded (about 2^22 sleeps); one that runs out raises the workgroup's abort
// flag and bit 2 of the info word, every other wait then gives up too, and
// all waves exit.
constexpr int FUSED_MTP = 16;                 // tile-column pairs per block (mt <= 32)
struct FusedSlot {
  int seq, state;                             // state: 0 free, 1 block, 2 end of queue
  int blk, link, diag;
  int cols[FUSED_MTP];                        // off-diagonal wave tiles done per column pair
  unsigned long long dmax;                    // bits of the largest diagonal entry (>= 0)
};
struct FusedCtl {
  FusedSlot slot[2];
  int fbar;                                   // factor-team barrier arrivals
  int abort;
};

__device__ __forceinline__ int lds_ld(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(int* p, int v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); }
__device__ __forceinline__ void wg_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); }

// Waits (the whole wave) until cond() holds; false if the wait ran out or the
// workgroup aborted.  A wait that runs out raises the abort flag.
template <class F>
__device__ __forceinline__ bool fused_wait(FusedCtl* ctl, DevInfo* info, F cond) {
  for (int it = 0; it < (1 << 22); ++it) {
    if (cond()) {
      wg_acquire();
      return true;
    }
    if (lds_ld(&ctl->abort)) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  if ((threadIdx.x & 63) == 0) {
    lds_st(&ctl->abort, 1);
    atomicOr(&info->nonfinite, 2);
  }
  return false;
}

// The factor team's synchronization inside the fused kernel.
struct TeamSync {
  static constexpr bool kPrefetch = false;   // the SYRK team's tiles are still in L2
  FusedCtl* ctl;
  FusedSlot* slot;
  DevInfo* info;
  int gen;     // barrier arrivals this wave has waited for
  int mtp;     // tile-column pairs of the block
  bool ok;
  __device__ __forceinline__ void sync() {
    wg_release();
    if ((threadIdx.x & 63) == 0) lds_add(&ctl->fbar, 1);
    gen += 4;
    const int g = gen;
    int* bar = &ctl->fbar;
    if (!fused_wait(ctl, info, [&]() { return lds_ld(bar) >= g; })) ok = false;
  }
  // panel c0 (tile columns c0, c0 + 1) needs the off-diagonal wave tiles of
  // column pair c0 / 2: pairs below it, mtp - 1 - c0 / 2 of them
  __device__ __forceinline__ bool wait_panel(int c0) {
    if (!ok) return false;
    const int q = c0 >> 1, need = mtp - 1 - q;
    int* cnt = &slot->cols[q];
    ok = fused_wait(ctl, info, [&]() { return lds_ld(cnt) >= need; });
    return ok;
  }
};

// One 32x32 wave tile (tile rows 2R, 2R+1, tile columns 2C, 2C+1) of block b's
// M_i = A_i D_i A_i' (+ delta I), by one wave with operands loaded straight
// from memory (two K steps in flight).  The per-tile products and their order
// are those of k_syrk.  Returns the largest real diagonal entry it stored
// (0 off the diagonal).
template <typename T>
__device__ __forceinline__ double syrk_wave_tile(const BlockInfo& b, int R, int C,
                                                 const T* __restrict__ A,
                                                 const double* __restrict__ Dp,
                                                 T* __restrict__ LB, double delta) {
  const int lane = threadIdx.x & 63;
  const int I0 = 2 * R, J0 = 2 * C;
  bool use[2][2];
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc)
      use[tr][tc] = I0 + tr < b.mt && J0 + tc < b.mt && I0 + tr >= J0 + tc;
  const T* rp[2];
  const T* cp[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    rp[u] = A + a_tile(b, min(I0 + u, b.mt - 1), 0) + lane;
    cp[u] = A + a_tile(b, min(J0 + u, b.mt - 1), 0) + lane;
  }
  const double* dp = Dp + b.dpoff + (lane >> 4);
  typedef typename Acc<T>::type AT;
  AT acc[2][2];
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc) acc[tr][tc] = AT{0, 0, 0, 0};
  struct Stage { T a[2][4], c[2][4]; double d[4]; };
  auto load = [&](int K, Stage& S) {
    const long long o = (long long)min(K, b.nt - 1) * TE;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        S.a[u][s] = rp[u][o + 64 * s];
        S.c[u][s] = cp[u][o + 64 * s];
      }
#pragma unroll
    for (int s = 0; s < 4; ++s) S.d[s] = dp[(long long)min(K, b.nt - 1) * TS + 4 * s];
  };
  auto step = [&](const Stage& S) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const T dd = (T)S.d[s];
      const T b0 = S.c[0][s] * dd, b1 = S.c[1][s] * dd;
      if (use[0][0]) acc[0][0] = mfma(S.a[0][s], b0, acc[0][0]);
      if (use[0][1]) acc[0][1] = mfma(S.a[0][s], b1, acc[0][1]);
      if (use[1][0]) acc[1][0] = mfma(S.a[1][s], b0, acc[1][0]);
      if (use[1][1]) acc[1][1] = mfma(S.a[1][s], b1, acc[1][1]);
    }
  };
  Stage S0, S1;
  load(0, S0);
  load(1, S1);
  for (int K = 0; K < b.nt; K += 2) {
    step(S0);
    load(K + 2, S0);
    if (K + 1 < b.nt) step(S1);
    load(K + 3, S1);
  }
  double dmax = 0.0;
#pragma unroll
  for (int tr = 0; tr < 2; ++tr) {
#pragma unroll
    for (int tc = 0; tc < 2; ++tc) {
      const int I = I0 + tr, J = J0 + tc;
      if (!use[tr][tc]) continue;
      T* dst = LB + lb_tile(b, I, J);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = acc[tr][tc][r];
        const int i = acc_row<T>(lane, r), j = lane & 15;
        if (I == J && i == j) {
          const bool real = TS * I + i < b.m;
          v = real ? (T)(v + delta) : T(1);
          if (real) dmax = fmax(dmax, (double)v);
        }
        dst[acc_index<T>(lane, r)] = v;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  return dmax;
}

template <typename T, int BF_RMAX>
__global__ __launch_bounds__(512, 1) void k_factor_fused(
    const BlockInfo* __restrict__ blk, const int* __restrict__ order, int nblk,
    int* __restrict__ queue, int nb, const T* __restrict__ Aw, const double* __restrict__ A,
    const double* __restrict__ C, const int* __restrict__ lptr, const int* __restrict__ lcol,
    const double* __restrict__ lval, const double* __restrict__ Dp, T* __restrict__ LB,
    T* __restrict__ LINV, double* __restrict__ PQ, double delta, DevInfo* info) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ FusedCtl ctl;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid == 0) {
    for (int s2 = 0; s2 < 2; ++s2) {
      ctl.slot[s2].seq = s2 - 2;
      ctl.slot[s2].state = 0;
    }
    ctl.fbar = 0;
    ctl.abort = 0;
  }
  __syncthreads();   // the only workgroup barrier: both teams pass it once

  if (wave >= 4) {
    // ---------------- SYRK team
    const int sw = wave - 4;
    for (int k = 0;; ++k) {
      FusedSlot* sl = &ctl.slot[k & 1];
      if (sw == 0) {
        // the leader takes the slot once its previous block (k - 2) is done;
        // the other waves wait for the slot's new sequence number only (the
        // leader may already have moved it on when they get here)
        if (!fused_wait(&ctl, info, [&]() { return lds_ld(&sl->seq) == k - 2 && lds_ld(&sl->state) == 0; }))
          return;
        int g = 0;
        if (lane == 0) g = atomicAdd(queue, 1);
        g = __shfl(g, 0);
        if (lane == 0) {
          if (g < nblk) {
            sl->blk = order[g];
            sl->link = 0;
            sl->diag = 0;
            for (int q = 0; q < FUSED_MTP; ++q) sl->cols[q] = 0;
            sl->dmax = 0ull;
          }
          lds_st(&sl->state, g < nblk ? 1 : 2);
        }
        // the slot's fields before its sequence number
        wg_release();
        if (lane == 0) lds_st(&sl->seq, k);
      }
      if (!fused_wait(&ctl, info, [&]() { return lds_ld(&sl->seq) == k; })) return;
      if (lds_ld(&sl->state) == 2) return;
      const BlockInfo b = blk[sl->blk];
      // link columns: the team's 256 threads take the tile rows in turn
      for (int rr = 0; rr < b.kt; ++rr)
        link_tile_row<T>(b, rr, tid - 256, nb, A, C, lptr, lcol, lval, Dp, LB, PQ);
      wg_release();
      if (lane == 0) lds_add(&sl->link, 1);
      // diagonal wave tiles, then the off-diagonal ones by column pair
      const int MT = (b.mt + 1) >> 1;
      for (int R = sw; R < MT; R += 4) {
        const double dm = syrk_wave_tile<T>(b, R, R, Aw, Dp, LB, delta);
        if (lane == 0) atomicMax(&sl->dmax, (unsigned long long)__double_as_longlong(dm));
        wg_release();
        if (lane == 0) lds_add(&sl->diag, 1);
      }
      int e = 0;
      for (int Cq = 0; Cq < MT - 1; ++Cq)
        for (int R = Cq + 1; R < MT; ++R, ++e) {
          if ((e & 3) != sw) continue;
          syrk_wave_tile<T>(b, R, Cq, Aw, Dp, LB, delta);
          wg_release();
          if (lane == 0) lds_add(&sl->cols[Cq], 1);
        }
      if (lds_ld(&ctl.abort)) return;
    }
  } else {
    // ---------------- factor team
    TeamSync sy{&ctl, nullptr, info, 0, 0, true};
    for (int k = 0;; ++k) {
      FusedSlot* sl = &ctl.slot[k & 1];
      if (!fused_wait(&ctl, info, [&]() { return lds_ld(&sl->seq) == k; })) return;
      if (lds_ld(&sl->state) == 2) return;
      const BlockInfo b = blk[sl->blk];
      const int MT = (b.mt + 1) >> 1;
      if (!fused_wait(&ctl, info, [&]() { return lds_ld(&sl->link) >= 4 && lds_ld(&sl->diag) >= MT; }))
        return;
      const double dmax = __longlong_as_double((long long)sl->dmax);
      const double thr = PIVOT_REL * fmax(dmax, 0.0);
      sy.slot = sl;
      sy.mtp = MT;
      panel_factor<T, BF_RMAX, 4>(b, LB, LINV, PQ, info, smem_raw, thr, sy);
      if (!sy.ok) return;
      sy.sync();               // every factor wave is done with the slot
      if (!sy.ok) return;
      if (tid == 0) {
        wg_release();
        lds_st(&sl->state, 0);
      }
    }
  }
}

// ---------------------------------------------------------------- a5
// Schur contribution of block i: PQ = F D F' - X X' with X = W_i' (the
// bordered rows of the factor), in FP64 whatever the factor precision.
template <typename T>
__global__ __launch_bounds__(256) void k_schur_contrib(const BlockInfo* __restrict__ blk,
                                                       const int* __restrict__ order,
                                                       const T* __restrict__ LB,
                                                       double* __restrict__ PQ) {
  const int tid = threadIdx.x, lane = tid & 63;
  schur_rows<T>(blk[order[blockIdx.x]], LB, PQ, __builtin_amdgcn_readfirstlane(tid >> 6), lane);
}

// Element (q, q2) of block i's symmetric contribution (lower tiles stored).
__device__ inline double pq_get(const double* PQ, const BlockInfo& b, int q, int q2) {
  if ((q >> 4) < (q2 >> 4)) { int t = q; q = q2; q2 = t; }
  return PQ[pq_tile(b, q >> 4, q2 >> 4) + (q2 & 15) * TS + (q & 15)];
}

// One workgroup per link pair j: T_jj (col-major, + delta I), T_{j+1,j}
// (col-major) and E_j (l_j x nb, col-major; columns: the global rows, then
// x_0), each entry the fixed-order sum of its two contributing blocks (plus
// F0 in the x_0 columns), and the pivot threshold of the pair.
__global__ __launch_bounds__(256) void k_assemble_pairs(
    const BlockInfo* __restrict__ blk, int P, int nb, int n0, const int* __restrict__ lsz,
    const long long* __restrict__ tdoff, const long long* __restrict__ tooff,
    const long long* __restrict__ eoff, const double* __restrict__ PQ,
    const double* __restrict__ F0, const long long* __restrict__ loff, double delta,
    double* __restrict__ Td, double* __restrict__ To, double* __restrict__ E,
    double* __restrict__ thrT) {
  const int j = blockIdx.x;
  const BlockInfo bl = blk[j], br = blk[j + 1];
  const int l = lsz[j], ng = nb - n0;
  const int offR = TS * bl.ktL;          // pair j inside block j (its right section)
  const int x0l = TS * (bl.ktL + bl.ktR), x0r = TS * (br.ktL + br.ktR);
  __shared__ double s_max[4];
  double md = 0.0;
  for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
    const int a = idx % l, c = idx / l;
    double v = pq_get(PQ, bl, offR + a, offR + c) + pq_get(PQ, br, a, c);
    if (a == c) {
      v += delta;
      md = fmax(md, v);
    }
    Td[tdoff[j] + idx] = v;
  }
  if (j + 1 < P) {
    const int l2 = lsz[j + 1];
    const int offR2 = TS * br.ktL;
    for (int idx = threadIdx.x; idx < l2 * l; idx += blockDim.x) {
      const int a = idx % l2, c = idx / l2;
      To[tooff[j] + idx] = pq_get(PQ, br, offR2 + a, c);
    }
  }
  for (int idx = threadIdx.x; idx < l * nb; idx += blockDim.x) {
    const int a = idx % l, c = idx / l;
    double v = pq_get(PQ, bl, offR + a, x0l + c) + pq_get(PQ, br, a, x0r + c);
    if (F0 && c >= ng) v += F0[(loff[j] + a) * n0 + (c - ng)];
    E[eoff[j] + idx] = v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off));
  if (lane == 0) s_max[wave] = md;
  __syncthreads();
  if (threadIdx.x == 0)
    thrT[j] = PIVOT_REL * fmax(fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3])), 0.0);
}

// S00 (nb x nb; the global rows, then x_0) = K0's border + sum_i (F D F' -
// W'W)_i[border, border]: K0' holds delta I on the global rows, their x_0 part
// Wg0 (rows nl.. of the extended F0) off the diagonal, and -D_0^-1 on x_0.
// One workgroup per entry, each thread a fixed strided subset of the blocks,
// then a fixed reduction tree.
__global__ __launch_bounds__(256) void k_assemble_s00(const BlockInfo* __restrict__ blk, int N,
                                                      int nb, int n0, long long nl,
                                                      const double* __restrict__ PQ,
                                                      const double* __restrict__ D0,
                                                      const double* __restrict__ F0, double delta,
                                                      double* __restrict__ S00) {
  __shared__ double sh[4];
  const int idx = blockIdx.x;
  const int a = idx % nb, c = idx / nb, ng = nb - n0;
  if (c > a) return;   // lower triangle computed, mirrored below
  double v = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const BlockInfo& b = blk[i];
    const int x0 = TS * (b.ktL + b.ktR);
    v += pq_get(PQ, b, x0 + a, x0 + c);
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    if (a == c) t = a < ng ? delta : -1.0 / D0[a - ng];
    else if (a >= ng && c < ng && F0) t = F0[(nl + c) * n0 + (a - ng)];
    t += ((sh[0] + sh[1]) + (sh[2] + sh[3]));
    S00[a + c * nb] = t;
    S00[c + a * nb] = t;
  }
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

// FP32 shadow of the constraint blocks (FP32 mode).
__global__ void k_convert_f32(long long n, const double* __restrict__ src, float* __restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ------------------------------------------------------------- launchers
void launch_convert_f32(hipStream_t st, long long n, const double* src, float* dst) {
  long long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (n > 0) hipLaunchKernelGGL(k_convert_f32, dim3((int)g), dim3(256), 0, st, n, src, dst);
}

void launch_prep(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                 long long d0off, const double* x, const double* z, const double* q, double rho,
                 double* Dp, double* xs, double* zs, DevInfo* info) {
  hipLaunchKernelGGL(k_prep, dim3(N + 1), dim3(256), 0, st, blk, N, n0, x0off, d0off, x, z, q, rho,
                     Dp, xs, zs, info);
}

template <typename T>
void launch_syrk(hipStream_t st, const BlockInfo* blk, const int4* items, int nitems,
                 const T* A, const double* Dp, T* LB, double delta) {
  const int grid = 8 * ((nitems + 7) / 8);
  hipLaunchKernelGGL(k_syrk<T>, dim3(grid), dim3(256), 0, st, blk, items, nitems, A, Dp, LB,
                     delta);
}
template void launch_syrk<double>(hipStream_t, const BlockInfo*, const int4*, int, const double*,
                                  const double*, double*, double);
template void launch_syrk<float>(hipStream_t, const BlockInfo*, const int4*, int, const float*,
                                 const double*, float*, double);

template <typename T>
void launch_link(hipStream_t st, const BlockInfo* blk, const int2* items, int nitems, int nb,
                 const double* A, const double* C, const int* lptr, const int* lcol,
                 const double* lval, const double* Dp, T* LB, double* PQ) {
  if (nitems == 0) return;
  hipLaunchKernelGGL(k_link<T>, dim3(nitems), dim3(256), 0, st, blk, items, nb, A, C, lptr, lcol,
                     lval, Dp, LB, PQ);
}
template void launch_link<double>(hipStream_t, const BlockInfo*, const int2*, int, int,
                                  const double*, const double*, const int*, const int*,
                                  const double*, const double*, double*, double*);
template void launch_link<float>(hipStream_t, const BlockInfo*, const int2*, int, int,
                                 const double*, const double*, const int*, const int*,
                                 const double*, const double*, float*, double*);

// Panel kernel (it also forms the blocks' Schur contributions); workgroup w
// takes block order[w].  Four waves per block for bordered blocks of up to
// 4 BF_RMAX_MAX tile rows (five rows per wave up to 20, six up to 24), or
// eight waves (five rows each) for blocks of up to 8 * 5 tile rows.
template <typename T>
void launch_block_factor_panel(hipStream_t st, const BlockInfo* blk, const int* order, int n,
                               int max_rt, T* LB, T* LINV, double* PQ, DevInfo* info, int waves,
                               int max_kt) {
  if (n == 0) return;
  // LDS: the panel column (max_rt tiles), L_cc^-1, the diagonal tile and one
  // per-wave tile, at the form's leading dimension; then as many FP64
  // Schur-contribution tiles as fit beside it without lowering the
  // occupancy the launch bounds ask for (two four-wave workgroups or one
  // eight-wave workgroup per CU, of the CU's 160 KiB)
  const size_t tile = (size_t)TS * BfLd<5>::LD * sizeof(T);
  const size_t base = (size_t)(max_rt + 2 + waves) * tile;
  const size_t budget = (waves == 8 ? 156 : 78) * 1024;
  const size_t tile64 = (size_t)TS * BfLd<5>::LD * sizeof(double);
  int cap = 0;
  if (budget > base) cap = (int)((budget - base) / tile64);
  if (max_kt >= 0) cap = std::min(cap, max_kt * (max_kt + 1) / 2);
  const size_t shmem = base + (size_t)cap * tile64;
  if (waves == 8) {
    hipLaunchKernelGGL((k_block_factor_panel<T, 5, 8>), dim3(n), dim3(512), shmem, st, blk, order,
                       LB, LINV, PQ, info, cap);
  } else if (max_rt <= 20) {
    hipLaunchKernelGGL((k_block_factor_panel<T, 5, 4>), dim3(n), dim3(256), shmem, st, blk, order,
                       LB, LINV, PQ, info, cap);
  } else {
    hipLaunchKernelGGL((k_block_factor_panel<T, 6, 4>), dim3(n), dim3(256), shmem, st, blk, order,
                       LB, LINV, PQ, info, cap);
  }
}
// The fused launch over the panel bucket (blocks order[0, n), bordered tile
// rows at most max_rt <= 4 BF_RMAX_MAX, tile columns at most 2 FUSED_MTP):
// one eight-wave workgroup per CU (at most n).  queue: one int, zeroed here.
template <typename T>
void launch_factor_fused(hipStream_t st, const BlockInfo* blk, const int* order, int n,
                         int max_rt, int* queue, int nb, const T* Aw, const double* A,
                         const double* C, const int* lptr, const int* lcol, const double* lval,
                         const double* Dp, T* LB, T* LINV, double* PQ, double delta,
                         DevInfo* info, int num_cu) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, queue);
  const int grid = std::min(n, num_cu);
  if (max_rt <= 20) {
    const size_t shmem = (size_t)(max_rt + 6) * TS * BfLd<5>::LD * sizeof(T);
    hipLaunchKernelGGL((k_factor_fused<T, 5>), dim3(grid), dim3(512), shmem, st, blk, order, n,
                       queue, nb, Aw, A, C, lptr, lcol, lval, Dp, LB, LINV, PQ, delta, info);
  } else {
    const size_t shmem = (size_t)(max_rt + 6) * TS * BfLd<6>::LD * sizeof(T);
    hipLaunchKernelGGL((k_factor_fused<T, 6>), dim3(grid), dim3(512), shmem, st, blk, order, n,
                       queue, nb, Aw, A, C, lptr, lcol, lval, Dp, LB, LINV, PQ, delta, info);
  }
}
template void launch_factor_fused<double>(hipStream_t, const BlockInfo*, const int*, int, int, int*,
                                          int, const double*, const double*, const double*,
                                          const int*, const int*, const double*, const double*,
                                          double*, double*, double*, double, DevInfo*, int);
template void launch_factor_fused<float>(hipStream_t, const BlockInfo*, const int*, int, int, int*,
                                         int, const float*, const double*, const double*,
                                         const int*, const int*, const double*, const double*,
                                         float*, float*, double*, double, DevInfo*, int);
bool factor_fused_fits(int rt, int mt) { return rt <= 4 * BF_RMAX_MAX && mt <= 2 * FUSED_MTP; }

// Column-at-a-time kernel (any height), then the Schur contributions.
template <typename T>
void launch_block_factor_col(hipStream_t st, const BlockInfo* blk, const int* order, int n,
                             int max_rt, T* LB, T* LINV, double* PQ, DevInfo* info) {
  if (n == 0) return;
  const size_t shmem = (size_t)(max_rt + 1) * TS * (TS + 1) * sizeof(T);   // padded tiles
  hipLaunchKernelGGL(k_block_factor<T>, dim3(n), dim3(256), shmem, st, blk, order, LB, LINV, info);
  hipLaunchKernelGGL(k_schur_contrib<T>, dim3(n), dim3(256), 0, st, blk, order, LB, PQ);
}
bool block_factor_panel_fits(int rt) { return rt <= 4 * BF_RMAX_MAX; }
bool block_factor_panel8_fits(int rt) { return rt <= 8 * 5; }
template void launch_block_factor_panel<double>(hipStream_t, const BlockInfo*, const int*, int, int,
                                                double*, double*, double*, DevInfo*, int, int);
template void launch_block_factor_panel<float>(hipStream_t, const BlockInfo*, const int*, int, int,
                                               float*, float*, double*, DevInfo*, int, int);
template void launch_block_factor_col<double>(hipStream_t, const BlockInfo*, const int*, int, int,
                                              double*, double*, double*, DevInfo*);
template void launch_block_factor_col<float>(hipStream_t, const BlockInfo*, const int*, int, int,
                                             float*, float*, double*, DevInfo*);

void launch_assemble(hipStream_t st, const BlockInfo* blk, int N, int nb, int n0, long long nl,
                     const int* lsz, const long long* tdoff, const long long* tooff,
                     const long long* eoff, const double* PQ, const double* F0L,
                     const double* F0, const long long* loff, double delta, const double* D0,
                     double* Td, double* To, double* E, double* S00, double* thrT) {
  const int P = N - 1;
  if (P > 0)
    hipLaunchKernelGGL(k_assemble_pairs, dim3(P), dim3(256), 0, st, blk, P, nb, n0, lsz, tdoff,
                       tooff, eoff, PQ, F0L, loff, delta, Td, To, E, thrT);
  if (nb > 0)
    hipLaunchKernelGGL(k_assemble_s00, dim3(nb * nb), dim3(256), 0, st, blk, N, nb, n0, nl, PQ,
                       D0, F0, delta, S00);
}

}  // namespace ahlp
