// Solve phase (a7) and interior-point glue (a8): products with the constraint
// operator, per-block substitutions with the bordered factors, assembly of the
// Schur right-hand side, elementwise updates and deterministic reductions.
//
// Vectors come in two layouts.  Canonical (the ABI's): x = [x_blocks, x_0],
// y = [y_blocks, y_L].  Padded (internal): every block padded to whole tiles,
// x_0 and block rows likewise, so tile products need no bounds checks.
#include "common.h"
#include "kernels.h"

namespace ahlp {

// ------------------------------------------------------------ layouts
// x-space: block i at dpoff (16 nt slots), x_0 at d0off (n0p slots).
__global__ void k_pad_x(const BlockInfo* __restrict__ blk, int N, int n0, long long x0off,
                        long long d0off, const double* __restrict__ x, double* __restrict__ xp,
                        const double* __restrict__ scale) {
  const int i = blockIdx.x;
  long long xo, po;
  int n, np;
  if (i < N) { xo = blk[i].xoff; po = blk[i].dpoff; n = blk[i].n; np = TS * blk[i].nt; }
  else { xo = x0off; po = d0off; n = n0; np = (n0 + TS - 1) / TS * TS; }
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    double v = 0.0;
    if (c < n) v = x[xo + c] * (scale ? scale[po + c] : 1.0);
    xp[po + c] = v;
  }
}

// y-space block rows: block i at voff (16 mt slots).
__global__ void k_pad_y(const BlockInfo* __restrict__ blk, const double* __restrict__ y,
                        double* __restrict__ yp) {
  const BlockInfo b = blk[blockIdx.x];
  for (int r = threadIdx.x; r < TS * b.mt; r += blockDim.x)
    yp[b.voff + r] = (r < b.m) ? y[b.yoff + r] : 0.0;
}

// rhx = rx - rz / x (canonical) and vx = D * rhx (padded).
__global__ void k_rhx(const BlockInfo* __restrict__ blk, int N, int n0, long long x0off,
                      long long d0off, const double* __restrict__ rx,
                      const double* __restrict__ rz, const double* __restrict__ xs,
                      const double* __restrict__ Dp, double* __restrict__ rhx,
                      double* __restrict__ vx) {
  const int i = blockIdx.x;
  long long xo, po;
  int n, np;
  if (i < N) { xo = blk[i].xoff; po = blk[i].dpoff; n = blk[i].n; np = TS * blk[i].nt; }
  else { xo = x0off; po = d0off; n = n0; np = (n0 + TS - 1) / TS * TS; }
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    double v = 0.0;
    if (c < n) {
      const double h = rx[xo + c] - rz[xo + c] / xs[xo + c];
      rhx[xo + c] = h;
      v = Dp[po + c] * h;
    }
    vx[po + c] = v;
  }
}

// ------------------------------------------------------------ block rows
// Row pass over the dense blocks for up to RV_MAX vectors at once (A is read
// once):  out_k = base_k + alpha_k (A_i v_k,i [+ C_i v_k,0]).
// One 16-row tile panel per wave.  A is read in 16-byte nontemporal pairs: lane l holds
// rows 2(l%8), 2(l%8)+1 of tile columns l/8 and 8 + l/8, so a tile costs two
// loads per lane; the partial sums are reduced over l/8.
template <int NV>
__global__ __launch_bounds__(256) void k_rows_nv(const BlockInfo* __restrict__ blk,
                                                 const int2* __restrict__ rowtiles, int nrt,
                                                 const double* __restrict__ A,
                                                 const double* __restrict__ C, long long d0off,
                                                 RowsArgs ra) {
  const int wt = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wt >= nrt) return;
  const int lane = threadIdx.x & 63, cb = lane >> 3, r2 = 2 * (lane & 7);
  const int2 rt = rowtiles[wt];
  const BlockInfo b = blk[rt.x];
  const int I = rt.y;
  double acc[NV][2];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k][0] = acc[k][1] = 0.0;
  const dv2* At = reinterpret_cast<const dv2*>(A + a_tile(b, I, 0));
#pragma unroll 4
  for (int K = 0; K < b.nt; ++K) {
    const dv2 a0 = ld_stream2(At + K * 128 + lane), a1 = ld_stream2(At + K * 128 + 64 + lane);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double* xv = ra.v[k] + b.dpoff + K * TS;
      const double x0 = xv[cb], x1 = xv[8 + cb];
      acc[k][0] += a0.x * x0 + a1.x * x1;
      acc[k][1] += a0.y * x0 + a1.y * x1;
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (!ra.with_C[k]) continue;
    const double* x0v = ra.v[k] + d0off;
    for (int Q = 0; Q < b.kc0; ++Q) {
      const dv2* ct = reinterpret_cast<const dv2*>(C + c_tile(b, I, Q));
      const dv2 a0 = ld_stream2(ct + lane), a1 = ld_stream2(ct + 64 + lane);
      const double x0 = x0v[Q * TS + cb], x1 = x0v[Q * TS + 8 + cb];
      acc[k][0] += a0.x * x0 + a1.x * x1;
      acc[k][1] += a0.y * x0 + a1.y * x1;
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v = acc[k][h];
      v += __shfl_xor(v, 8);
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      acc[k][h] = v;
    }
  if (lane < 8) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = TS * I + r2 + h;
      const bool in = row < b.m;
      double prev = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        double base = 0.0;
        if (ra.chain[k]) base = prev;
        else if (ra.base[k] && in) base = ra.base[k][b.yoff + row];
        const double v = in ? base + ra.alpha[k] * acc[k][h] : 0.0;
        prev = v;
        if (ra.padded[k]) ra.out[k][b.voff + row] = v;
        else if (in) ra.out[k][b.yoff + row] = v;
      }
    }
  }
}

// The dual rows after the blocks, out = base + alpha * (F xp [+ F0 x0]),
// 256 threads per workgroup: the link rows, out[pair j, row a] = base + alpha
// (FR_j xp_j + FL_j xp_{j+1} [+ F0 x0]), a pair per workgroup (its first wave)
// in the first gridP workgroups; then global row k by workgroup gridP + k,
// out[nl + k] = base +
// alpha (sum_i Wg_i xp_i [+ Wg0 x0]), its entries kept as one compressed row
// over the padded x (gptr, gidx, gval): each thread a fixed strided share,
// then a fixed reduction tree.  F0 (when given) is the extended (nl + ng) x n0
// coupling; F0L the same pointer, or null when the link rows' part of it is
// zero.
__device__ double block_reduce(int op, double v);
__global__ __launch_bounds__(256) void k_linkrows(
    const BlockInfo* __restrict__ blk, int P, int gridP, int n0, const int* __restrict__ lsz,
    const long long* __restrict__ loff, long long nl, const int* __restrict__ lptr,
    const int* __restrict__ lcol, const double* __restrict__ lval, const int* __restrict__ gptr,
    const int* __restrict__ gidx, const double* __restrict__ gval, const double* __restrict__ xp,
    const double* __restrict__ x0, const double* __restrict__ F0, const double* __restrict__ F0L,
    const double* __restrict__ base, double alpha, double* __restrict__ out) {
  if ((int)blockIdx.x >= gridP) {
    const int k = blockIdx.x - gridP;
    double v = 0.0;
    const int e1 = gptr[k + 1];
    for (int e = gptr[k] + threadIdx.x; e < e1; e += blockDim.x) v += gval[e] * xp[gidx[e]];
    if (F0 && x0)
      for (int c = threadIdx.x; c < n0; c += blockDim.x) v += F0[(nl + k) * n0 + c] * x0[c];
    const double t = block_reduce(0, v);
    if (threadIdx.x == 0) out[nl + k] = (base ? base[nl + k] : 0.0) + alpha * t;
    return;
  }
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  for (int j = blockIdx.x; j < P; j += gridP) {
    const BlockInfo bl = blk[j], br = blk[j + 1];
    const int l = lsz[j];
    for (int a = lane; a < l; a += 64) {
      double s = 0.0;
      const int qr = TS * bl.ktL + a;   // right section of block j
      for (int e = lptr[bl.csr_off + qr]; e < lptr[bl.csr_off + qr + 1]; ++e)
        s += lval[e] * xp[bl.dpoff + lcol[e]];
      for (int e = lptr[br.csr_off + a]; e < lptr[br.csr_off + a + 1]; ++e)
        s += lval[e] * xp[br.dpoff + lcol[e]];
      if (F0L && x0)
        for (int c = 0; c < n0; ++c) s += F0L[(loff[j] + a) * n0 + c] * x0[c];
      const long long o = loff[j] + a;
      out[o] = (base ? base[o] : 0.0) + alpha * s;
    }
  }
}

// ------------------------------------------------------------ block columns
// g = A_i' yp_i + F_i' yL for one 16-column tile per wave, then by mode:
//   0: out = g          1: out = cvec - g - zvec       2: out = D (g - rhx)
// gout (optional) receives g.
__global__ __launch_bounds__(256) void k_cols(const BlockInfo* __restrict__ blk,
                                              const int2* __restrict__ coltiles, int nct,
                                              const double* __restrict__ A,
                                              const double* __restrict__ yp,
                                              const double* __restrict__ yL,
                                              const int* __restrict__ cptr,
                                              const int* __restrict__ crow,
                                              const double* __restrict__ cval, int mode,
                                              const double* __restrict__ cvec,
                                              const double* __restrict__ zvec,
                                              const double* __restrict__ Dp,
                                              double* __restrict__ gout,
                                              double* __restrict__ out,
                                              const DzArgs dzv) {
  const int wt = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wt >= nct) return;
  const int lane = threadIdx.x & 63, cb = lane >> 3, r2 = 2 * (lane & 7);
  const int2 ct = coltiles[wt];
  const BlockInfo b = blk[ct.x];
  const int K = ct.y;
  double acc0 = 0.0, acc1 = 0.0;   // tile columns cb and 8 + cb
  const double* yb = yp + b.voff + r2;
#pragma unroll 8
  for (int I = 0; I < b.mt; ++I) {
    const dv2* tile = reinterpret_cast<const dv2*>(A + a_tile(b, I, K));
    const dv2 a0 = ld_stream2(tile + lane), a1 = ld_stream2(tile + 64 + lane);
    const double2 yv = *reinterpret_cast<const double2*>(yb + I * TS);
    acc0 += a0.x * yv.x + a0.y * yv.y;
    acc1 += a1.x * yv.x + a1.y * yv.y;
  }
#pragma unroll
  for (int sft = 1; sft < 8; sft <<= 1) {
    acc0 += __shfl_xor(acc0, sft);
    acc1 += __shfl_xor(acc1, sft);
  }
  if ((lane & 7) == 0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = TS * K + cb + 8 * h;
      if (col >= b.n) continue;
      double g = h ? acc1 : acc0;
      for (int e = cptr[b.csc_off + col]; e < cptr[b.csc_off + col + 1]; ++e)
        g += cval[e] * yL[crow[e]];
      const long long o = b.xoff + col;
      if (gout) gout[o] = g;
      double v = g;
      if (mode == 1) v = cvec[o] - g - zvec[o];
      else if (mode == 2) v = Dp[b.dpoff + col] * (g - cvec[o]);
      if (out) out[o] = v;
      if (dzv.dz) dzv.dz[o] = (dzv.rz[o] - dzv.zs[o] * v) / dzv.xs[o];
    }
  }
}

// Per-block partial sums C_i' yp_i: one 16-column tile of C_i per wave.
__global__ __launch_bounds__(256) void k_ccols(const BlockInfo* __restrict__ blk,
                                               const int2* __restrict__ ctiles, int nctile, int n0,
                                               const double* __restrict__ C,
                                               const double* __restrict__ yp,
                                               double* __restrict__ part) {
  const int wt = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wt >= nctile) return;
  const int lane = threadIdx.x & 63, cb = lane >> 3, r2 = 2 * (lane & 7);
  const int2 ct = ctiles[wt];
  const BlockInfo b = blk[ct.x];
  const int Q = ct.y;
  double acc0 = 0.0, acc1 = 0.0;
  const double* yb = yp + b.voff + r2;
#pragma unroll 8
  for (int I = 0; I < b.mt; ++I) {
    const dv2* tile = reinterpret_cast<const dv2*>(C + c_tile(b, I, Q));
    const dv2 a0 = ld_stream2(tile + lane), a1 = ld_stream2(tile + 64 + lane);
    const double2 yv = *reinterpret_cast<const double2*>(yb + I * TS);
    acc0 += a0.x * yv.x + a0.y * yv.y;
    acc1 += a1.x * yv.x + a1.y * yv.y;
  }
#pragma unroll
  for (int sft = 1; sft < 8; sft <<= 1) {
    acc0 += __shfl_xor(acc0, sft);
    acc1 += __shfl_xor(acc1, sft);
  }
  if ((lane & 7) == 0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = TS * Q + cb + 8 * h;
      if (col < n0) part[(long long)ct.x * n0 + col] = h ? acc1 : acc0;
    }
  }
}

// g0[c] = sum_i part[i][c] + (F0' yL)[c] with one workgroup per column: each
// thread sums a fixed strided subset, then a fixed tree; then by mode as k_cols.
__device__ double block_reduce(int op, double v);
__global__ __launch_bounds__(256) void k_x0_sum(int N, int n0, long long nl, long long f0first,
                                                const double* __restrict__ part,
                                                const double* __restrict__ F0,
                                                const double* __restrict__ yL, int mode,
                                                const double* __restrict__ cvec,
                                                const double* __restrict__ zvec, long long x0off,
                                                double* __restrict__ gout,
                                                double* __restrict__ out) {
  const int c = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) v += part[(long long)i * n0 + c];
  if (F0)
    for (long long r = f0first + threadIdx.x; r < nl; r += blockDim.x) v += F0[r * n0 + c] * yL[r];
  const double g = block_reduce(0, v);
  if (threadIdx.x == 0) {
    const long long o = x0off + c;
    if (gout) gout[o] = g;
    if (out) out[o] = (mode == 1) ? cvec[o] - g - zvec[o] : g;
  }
}

// ------------------------------------------------------------ substitutions
// The block solves walk the mt tile columns of L_i in a dependent chain; the
// tiles a step reads do not depend on the chain, so each step loads the next
// step's tiles into registers (two register sets, alternating) while it
// works.  BS_PF tiles of a column per wave are held (rows p+1+w, p+5+w, ...);
// rows beyond them, in blocks with more than 4 BS_PF bordered tile rows below
// the diagonal, are loaded in place.  Loads past either end (column mt after
// the last forward step, column -1 after the last backward one, rows past
// rt) are clamped to a valid tile and not used.
constexpr int BS_PF = 5;

template <typename T>
struct ColRegs {
  T t[BS_PF][4];   // tiles (p+1+w+4q, p), element 64 k + lane
  T li[4];         // inverted diagonal tile p
};

template <typename T>
__device__ __forceinline__ void load_col(const BlockInfo& b, const T* __restrict__ LB,
                                         const T* __restrict__ LINV, int p, int wave, int lane,
                                         ColRegs<T>& c) {
  const int pc = max(min(p, b.mt - 1), 0);
#pragma unroll
  for (int q = 0; q < BS_PF; ++q) {
    const int r = max(min(p + 1 + wave + 4 * q, b.rt - 1), pc);
    const T* L = LB + lb_tile(b, r, pc);
#pragma unroll
    for (int k = 0; k < 4; ++k) c.t[q][k] = L[64 * k + lane];
  }
  const T* Li = LINV + b.linvoff + (long long)pc * TE;
#pragma unroll
  for (int k = 0; k < 4; ++k) c.li[k] = Li[64 * k + lane];
}

// Forward substitution with the bordered factor of block i: v = L_i^-1 t and,
// on the bordered rows, qn = -W_i' v.  t is read from tin (padded block-row
// vector) and v written to tv (tin may equal tv).
template <typename T>
__global__ __launch_bounds__(256) void k_block_fwd(const BlockInfo* __restrict__ blk,
                                                   const T* __restrict__ LB,
                                                   const T* __restrict__ LINV,
                                                   const double* __restrict__ tin,
                                                   double* __restrict__ tv,
                                                   double* __restrict__ qn) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* t = reinterpret_cast<double*>(smem_raw);
  const BlockInfo b = blk[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nr = TS * b.rt, nm = TS * b.mt;
  for (int r = tid; r < nr; r += blockDim.x) t[r] = (r < nm) ? tin[b.voff + r] : 0.0;
  // step p with the tiles in c; the next step's go to n
  auto step = [&](int p, const ColRegs<T>& c, ColRegs<T>& n) {
    load_col(b, LB, LINV, p + 1, wave, lane, n);
    __syncthreads();
    if (wave == 0) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += (double)c.li[k] * t[TS * p + 4 * k + (lane >> 4)];
      s = col_sum4(s);
      // all lanes have read t[p-block]; lanes 0..15 now overwrite it
      if (lane < 16) t[TS * p + lane] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BS_PF; ++q) {
      const int r = p + 1 + wave + 4 * q;
      if (r < b.rt) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) s += (double)c.t[q][k] * t[TS * p + 4 * k + (lane >> 4)];
        s = col_sum4(s);
        if (lane < 16) t[TS * r + lane] -= s;
      }
    }
    for (int r = p + 1 + wave + 4 * BS_PF; r < b.rt; r += 4) {
      const T* L = LB + lb_tile(b, r, p);
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) s += (double)L[64 * k + lane] * t[TS * p + 4 * k + (lane >> 4)];
      s = col_sum4(s);
      if (lane < 16) t[TS * r + lane] -= s;
    }
  };
  ColRegs<T> ra, rb;
  load_col(b, LB, LINV, 0, wave, lane, ra);
  for (int p = 0; p < b.mt; p += 2) {
    step(p, ra, rb);
    if (p + 1 < b.mt) step(p + 1, rb, ra);
  }
  __syncthreads();
  for (int r = tid; r < nm; r += blockDim.x) tv[b.voff + r] = t[r];
  for (int r = nm + tid; r < nr; r += blockDim.x) qn[b.qoff + (r - nm)] = t[r];
}

// Backward substitution: y = L_i^-T (v - W_i u_i), where u_i (the block's view
// of the Schur solution: left pair, right pair, x_0) fills the bordered rows.
// Writes dy (canonical) and the padded copy dyp.
template <typename T>
__global__ __launch_bounds__(256) void k_block_bwd(const BlockInfo* __restrict__ blk, int nb,
                                                   long long nl, const T* __restrict__ LB,
                                                   const T* __restrict__ LINV,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ u,
                                                   double* __restrict__ dy,
                                                   double* __restrict__ dyp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* y = reinterpret_cast<double*>(smem_raw);
  __shared__ double part[4][TS];
  const BlockInfo b = blk[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nr = TS * b.rt, nm = TS * b.mt;
  for (int r = tid; r < nr; r += blockDim.x) {
    double val;
    if (r < nm) {
      val = v[b.voff + r];
    } else {
      int qi;
      bool real;
      const int sec = link_section(b, r - nm, &qi, nb, &real);
      val = 0.0;
      if (real) {
        if (sec == 0) val = u[b.loffL + qi];
        else if (sec == 1) val = u[b.loffR + qi];
        else val = u[nl + qi];
      }
    }
    y[r] = val;
  }
  auto step = [&](int p, const ColRegs<T>& c, ColRegs<T>& n) {
    load_col(b, LB, LINV, p - 1, wave, lane, n);
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < BS_PF; ++q) {
      const int r = p + 1 + wave + 4 * q;
      if (r < b.rt) {
        const double yv = y[TS * r + (lane & 15)];
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s] += (double)c.t[q][s] * yv;
      }
    }
    for (int r = p + 1 + wave + 4 * BS_PF; r < b.rt; r += 4) {
      const T* L = LB + lb_tile(b, r, p);
      const double yv = y[TS * r + (lane & 15)];
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] += (double)L[64 * s + lane] * yv;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double x = row_sum16(acc[s]);
      if ((lane & 15) == 0) part[wave][4 * s + (lane >> 4)] = x;
    }
    __syncthreads();
    if (wave == 0) {
      // w = v_p - sum over waves (fixed order); y_p = Linv_p' w
      const int kcol = lane & 15;
      const double w = y[TS * p + kcol] - (part[0][kcol] + part[1][kcol] + part[2][kcol] + part[3][kcol]);
      // element (i, k) of Linv at 64 s + l:  i = l%16, k = 4 s + l/16;  y_p[k] = sum_i Linv[i][k] w[i]
      double s4[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        // this lane's w is w[lane % 16], the row index i it needs
        s4[s] = row_sum16((double)c.li[s] * w);
      }
      if ((lane & 15) == 0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) part[0][4 * s + (lane >> 4)] = s4[s];
      }
    }
    __syncthreads();
    if (tid < TS) y[TS * p + tid] = part[0][tid];
  };
  ColRegs<T> ra, rb;
  load_col(b, LB, LINV, b.mt - 1, wave, lane, ra);
  for (int p = b.mt - 1; p >= 0; p -= 2) {
    step(p, ra, rb);
    if (p >= 1) step(p - 1, rb, ra);
  }
  __syncthreads();
  for (int r = tid; r < nm; r += blockDim.x) {
    dyp[b.voff + r] = (r < b.m) ? y[r] : 0.0;
    if (r < b.m) dy[b.yoff + r] = y[r];
  }
}

// Schur right-hand side (Alg. 3): s_L[pair j] += qn_j[right section] +
// qn_{j+1}[left section]; the border (global rows, then x_0): s_b += sum_i
// qn_i[border section] (fixed order), on top of the global rows' part s_b
// already holds (b < ng) or of rhx_0 (x_0 entries).  Blocks below npb handle
// pairs, the next nb blocks one border entry each.
__global__ __launch_bounds__(256) void k_schur_rhs(const BlockInfo* __restrict__ blk, int N, int nb,
                                                   const int* __restrict__ lsz,
                                                   const long long* __restrict__ loff, long long nl,
                                                   int npb, const double* __restrict__ qn,
                                                   const double* __restrict__ rhx0,
                                                   double* __restrict__ s) {
  const int P = N - 1;
  if ((int)blockIdx.x < npb) {
    for (int j = blockIdx.x; j < P; j += npb) {
      const BlockInfo bl = blk[j], br = blk[j + 1];
      for (int a = threadIdx.x; a < lsz[j]; a += blockDim.x)
        s[loff[j] + a] += qn[bl.qoff + TS * bl.ktL + a] + qn[br.qoff + a];
    }
    return;
  }
  const int c = blockIdx.x - npb;
  double v = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const BlockInfo& b = blk[i];
    v += qn[b.qoff + TS * (b.ktL + b.ktR) + c];
  }
  const double t = block_reduce(0, v);
  const int ng = blk[0].ng;
  if (threadIdx.x == 0) s[nl + c] = (c < ng ? s[nl + c] : rhx0[c - ng]) + t;
}

// End of a solve for the x_0 columns and the link rows: g_0 = sum of the
// per-block partials C_i' dy_i + F0' dy_L (fixed order), dx_0 = u_0 and
// dz_0 = (rz_0 - z_0 dx_0) / x_0 (blocks below n0, one entry each); the
// remaining blocks copy the link part u_L of the Schur solution into dy.
__global__ __launch_bounds__(256) void k_solve_tail(int N, int n0, long long nl, long long f0first,
                                                    const double* __restrict__ part,
                                                    const double* __restrict__ F0,
                                                    const double* __restrict__ u, long long x0off,
                                                    long long mblk, double* __restrict__ gout,
                                                    double* __restrict__ dx, const DzArgs dzv,
                                                    double* __restrict__ dy) {
  if ((int)blockIdx.x < n0) {
    const int c = blockIdx.x;
    double v = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) v += part[(long long)i * n0 + c];
    if (F0)
      for (long long r = f0first + threadIdx.x; r < nl; r += blockDim.x) v += F0[r * n0 + c] * u[r];
    const double g = block_reduce(0, v);
    if (threadIdx.x == 0) {
      const long long o = x0off + c;
      gout[o] = g;
      const double d = u[nl + c];
      dx[o] = d;
      dzv.dz[o] = (dzv.rz[o] - dzv.zs[o] * d) / dzv.xs[o];
    }
    return;
  }
  const long long stride = (long long)(gridDim.x - n0) * blockDim.x;
  for (long long r = (long long)(blockIdx.x - n0) * blockDim.x + threadIdx.x; r < nl; r += stride)
    dy[mblk + r] = u[r];
}

// Refinement-check prologue, per block of x-space (and the x_0 segment):
// ex = rx - g - dz, ez = rz - zs dx - xs dz; xp = dx padded; w2p = D dx dz / x
// padded (if requested, zero on the x_0 segment).
__global__ void k_check_prep(const BlockInfo* __restrict__ blk, int N, int n0, long long x0off,
                             long long d0off, const double* __restrict__ rx,
                             const double* __restrict__ rz, const double* __restrict__ g,
                             const double* __restrict__ dx, const double* __restrict__ dz,
                             const double* __restrict__ xs, const double* __restrict__ zs,
                             const double* __restrict__ Dp, double* __restrict__ ex,
                             double* __restrict__ ez, double* __restrict__ xp,
                             double* __restrict__ w2p, const BndArgs b) {
  const int i = blockIdx.x;
  long long xo, po;
  int n, np;
  if (i < N) { xo = blk[i].xoff; po = blk[i].dpoff; n = blk[i].n; np = TS * blk[i].nt; }
  else { xo = x0off; po = d0off; n = n0; np = (n0 + TS - 1) / TS * TS; }
  const double smu = (b.ub && b.mode == 1) ? *b.smu : 0.0;
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    double v = 0.0, w = 0.0;
    if (c < n) {
      const long long o = xo + c;
      const double d = dx[o], e = dz[o];
      v = d;
      double exo = rx[o] - g[o] - e;
      double sw2 = 0.0;
      if (b.ub) {
        // ds = r_u - dx, dw = S^-1 (r_sw - W ds), r_sw = -SWe (predictor) or
        // smu - SWe - dS_aff dW_aff (corrector); zero off the bounded variables
        double ds = 0.0, dw = 0.0;
        if (isfinite(b.ub[o])) {
          const double sv = b.s[o], wv = b.w[o];
          ds = b.ru[o] - d;
          const double rsw = (b.mode == 1) ? smu - sv * wv - b.dsa[o] * b.dwa[o] : -sv * wv;
          dw = (rsw - wv * ds) / sv;
          sw2 = ds * dw / sv;
        }
        b.ds[o] = ds;
        b.dw[o] = dw;
      }
      if (b.q) exo += b.q[o] * d;
      if (i < N) w = Dp[po + c] * (d * e / xs[o] - sw2);
      ex[o] = exo;
      ez[o] = rz[o] - (zs[o] * d + xs[o] * e);
    }
    xp[po + c] = v;
    if (w2p) w2p[po + c] = w;
  }
}

// Residual-stage prologue, per block of x-space: rz_a = -x z; rhx = rd - rz_a / x;
// vx = D rhx, w1 = D / x (zero on the x_0 segment) and xp = x, all padded.
__global__ void k_resid_prep(const BlockInfo* __restrict__ blk, int N, int n0, long long x0off,
                             long long d0off, const double* __restrict__ x,
                             const double* __restrict__ z, const double* __restrict__ rd,
                             const double* __restrict__ xs, const double* __restrict__ Dp,
                             double* __restrict__ rzv, double* __restrict__ rhx,
                             double* __restrict__ vx, double* __restrict__ w1p,
                             double* __restrict__ xp, const BndArgs b,
                             double* __restrict__ rdt_out) {
  const int i = blockIdx.x;
  long long xo, po;
  int n, np;
  if (i < N) { xo = blk[i].xoff; po = blk[i].dpoff; n = blk[i].n; np = TS * blk[i].nt; }
  else { xo = x0off; po = d0off; n = n0; np = (n0 + TS - 1) / TS * TS; }
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    double hv = 0.0, w = 0.0, xv = 0.0;
    if (c < n) {
      const long long o = xo + c;
      xv = x[o];
      const double r = -xv * z[o];
      rzv[o] = r;
      double rdo = rd[o], sinv = 0.0;
      if (b.ub) {
        // the predictor's x right-hand side r_d + S^-1 (-SWe - W r_u)
        if (isfinite(b.ub[o])) {
          rdo -= b.w[o] + b.q[o] * b.ru[o];
          sinv = 1.0 / b.s[o];
        }
        rdt_out[o] = rdo;
      }
      const double h = rdo - r / xs[o];
      rhx[o] = h;
      hv = Dp[po + c] * h;
      if (i < N) w = Dp[po + c] * (1.0 / xs[o] - sinv);
    }
    vx[po + c] = hv;
    w1p[po + c] = w;
    xp[po + c] = xv;
  }
}

// ------------------------------------------------------------ elementwise
__global__ void k_axpy(long long n, double a, const double* __restrict__ x,
                       double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

// The transposed Newton matrix is a diagonal scaling of the Newton matrix:
// K' = diag(I, I, Z^-1) K diag(I, I, Z).  K' w = g is therefore solved as the
// Newton solve of (g_x, g_y, z g_z) followed by w_z = dz / z.  mode 0:
// out = z v; mode 1: out = v / z (may be in place).
__global__ void k_adj_scale(long long n, int mode, const double* __restrict__ zs,
                            const double* v, double* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = mode ? v[i] / zs[i] : zs[i] * v[i];
}

// dz = (rz - zs dx) / xs
__global__ void k_dz(long long n, const double* __restrict__ rz, const double* __restrict__ zs,
                     const double* __restrict__ xs, const double* __restrict__ dx,
                     double* __restrict__ dz) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dz[i] = (rz[i] - zs[i] * dx[i]) / xs[i];
}

// Refinement residual pieces in x-space: ex = rx - g - dz;  ez = rz - zs dx - xs dz.
// dual residual from a maintained g = A'y:  rd = c - g - z
__global__ void k_rd(long long n, const double* __restrict__ c, const double* __restrict__ g,
                     const double* __restrict__ z, double* __restrict__ rd) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    rd[i] = c[i] - g[i] - z[i];
}

__global__ void k_res_x(long long n, const double* __restrict__ rx, const double* __restrict__ rz,
                        const double* __restrict__ g, const double* __restrict__ dx,
                        const double* __restrict__ dz, const double* __restrict__ xs,
                        const double* __restrict__ zs, double* __restrict__ ex,
                        double* __restrict__ ez) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    ex[i] = rx[i] - g[i] - dz[i];
    ez[i] = rz[i] - (zs[i] * dx[i] + xs[i] * dz[i]);
  }
}

// w = D (a b) / x in padded x-space (a null: w = D / x); the x_0 part is zero.
__global__ void k_wscaled(const BlockInfo* __restrict__ blk, int N, int n0, long long x0off,
                          long long d0off, const double* __restrict__ a,
                          const double* __restrict__ b, const double* __restrict__ xs,
                          const double* __restrict__ Dp, double* __restrict__ w) {
  const int i = blockIdx.x;
  long long xo, po;
  int n, np;
  if (i < N) { xo = blk[i].xoff; po = blk[i].dpoff; n = blk[i].n; np = TS * blk[i].nt; }
  else { xo = x0off; po = d0off; n = 0; np = (n0 + TS - 1) / TS * TS; }
  for (int c = threadIdx.x; c < np; c += blockDim.x) {
    double v = 0.0;
    if (c < n) v = Dp[po + c] * (a ? a[xo + c] * b[xo + c] : 1.0) / xs[xo + c];
    w[po + c] = v;
  }
}

// out = t - smu a + b
__global__ void k_combine(long long n, const double* __restrict__ t, double smu,
                          const double* __restrict__ smu_dev, const double* __restrict__ a,
                          const double* __restrict__ b, double* __restrict__ out) {
  if (smu_dev) smu = *smu_dev;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (t[i] - smu * a[i]) + b[i];
}

// Mehrotra's centering target sigma mu = (mu_aff / mu)^3 mu from the reduction
// slots (sums x'z and (x + a_p dxa)'(z + a_d dza)), on the device so that the
// corrector needs no host value.  One thread.
__global__ void k_sigma_mu(double* __restrict__ scal, double inv_n, int s_xz, int s_muaff,
                           int s_out, int s_sw, int s_muaff_sw) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double xz = scal[s_xz], ma = scal[s_muaff];
  if (s_sw >= 0) {
    xz += scal[s_sw];
    ma += scal[s_muaff_sw];
  }
  const double mu = xz * inv_n;
  const double r = ma * inv_n / mu;
  scal[s_out] = r * r * r * mu;
}

// Right-hand side of a multiple centrality corrector (Gondzio): the
// complementarity products v at the trial point (x + at_p dx, z + at_d dz)
// moved into [beta_min, beta_max] sigma mu, a decrease capped at beta_max
// sigma mu: r = max(clip(v, lo, hi) - v, -hi), sigma mu from *smu.
__global__ void k_gondzio_rhs(long long n, const double* __restrict__ x,
                              const double* __restrict__ z, const double* __restrict__ dx,
                              const double* __restrict__ dz, double at_p, double at_d,
                              const double* __restrict__ smu, double beta_min, double beta_max,
                              double* __restrict__ r) {
  const double lo = beta_min * *smu, hi = beta_max * *smu;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (x[i] + at_p * dx[i]) * (z[i] + at_d * dz[i]);
    r[i] = fmax(fmin(fmax(v, lo), hi) - v, -hi);
  }
}

// Step x += min(1, eta * ratio) d with the ratio-test result on the device.
__global__ void k_steps(StepSet s, double eta) {
  const int v = blockIdx.y;
  const long long n = s.n[v];
  const double a = fmin(1.0, eta * *s.ratio[v]);
  const double* __restrict__ d = s.d[v];
  double* __restrict__ x = s.x[v];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] += a * d[i];
}

// Copy x0 part of the Schur solution into dx.
__global__ void k_copy(long long n, const double* __restrict__ src, double* __restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Predictor/corrector complementarity right-hand sides:
//   mode 0: rz = -x z;   mode 1: rz = sigma mu - x z - dxa dza  (sigma*mu in *smu)
__global__ void k_rz(long long n, int mode, const double* __restrict__ x,
                     const double* __restrict__ z, const double* __restrict__ dxa,
                     const double* __restrict__ dza, double sm, const double* __restrict__ sm_dev,
                     double* __restrict__ rz, const BndArgs b, double* __restrict__ rxc) {
  if (sm_dev) sm = *sm_dev;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double v = -x[i] * z[i];
    if (mode == 1) v += sm - dxa[i] * dza[i];
    rz[i] = v;
    if (rxc) {
      // the corrector's x right-hand side: rdt + S^-1 (smu - dS_aff dW_aff)
      double r = b.rdt[i];
      if (isfinite(b.ub[i])) r += (sm - b.dsa[i] * b.dwa[i]) / b.s[i];
      rxc[i] = r;
    }
  }
}

// ------------------------------------------------------------ bounds
__global__ void k_bnd_prep(long long n, const double* __restrict__ ub, const double* __restrict__ x,
                           const double* __restrict__ z, const double* __restrict__ s,
                           const double* __restrict__ w, double* __restrict__ ru,
                           double* __restrict__ q, double* __restrict__ zw, DevInfo* info) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double r = 0.0, qq = 0.0;
    const double wv = w[i];
    if (isfinite(ub[i])) {
      const double sv = s[i];
      if (!(sv > 0.0) || !(wv > 0.0) || !isfinite(sv) || !isfinite(wv)) bad = 1;
      r = ub[i] - x[i] - sv;
      qq = wv / sv;
    }
    ru[i] = r;
    q[i] = qq;
    zw[i] = z[i] - wv;
  }
  if (bad) atomicOr(&info->nonfinite, 1);
}
__global__ void k_bnd_start(long long n, const double* __restrict__ ub, const double* __restrict__ x,
                            double* __restrict__ z, double* __restrict__ s, double* __restrict__ w,
                            double* __restrict__ sm, double* __restrict__ wm) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    if (isfinite(ub[i])) {
      const double zv = z[i], sv = ub[i] - x[i], wv = fmax(-zv, 0.0);
      z[i] = fmax(zv, 0.0);
      s[i] = sv;
      w[i] = wv;
      sm[i] = sv;
      wm[i] = wv;
    } else {
      s[i] = 0.0;
      w[i] = 0.0;
      sm[i] = INFINITY;
      wm[i] = INFINITY;
    }
  }
}
__global__ void k_bnd_shift(long long n, const double* __restrict__ ub, double a, double c,
                            double* __restrict__ x, double* __restrict__ z, double* __restrict__ s,
                            double* __restrict__ w, double* __restrict__ sm,
                            double* __restrict__ wm) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    x[i] += a;
    z[i] += c;
    if (isfinite(ub[i])) {
      const double sv = s[i] + a, wv = w[i] + c;
      s[i] = sv;
      w[i] = wv;
      sm[i] = sv;
      wm[i] = wv;
    }
  }
}

__global__ void k_fill(long long n, double v, double* __restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = v;
}

__global__ void k_addscalar(long long n, double v, double* __restrict__ dst) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] += v;
}

// ------------------------------------------------------------ reductions
// Fixed grid and fixed per-thread ranges; partials reduced in a fixed tree.
// ops: 0 sum a*b, 1 max |a|, 2 min over b<0 of -a/b (inf if none),
//      3 sum (a + s1 b)(c + s2 d)  [mu_aff], 4 max (a + b), 5 min a,
//      6 min over b<0 of -a/b and over d<0 of -c/d
constexpr int RED_BLOCKS = RED_PARTIALS;
constexpr int RED_THREADS = 256;

__device__ inline double red_combine(int op, double x, double y) {
  return (op == 0 || op == 3) ? x + y : ((op == 2 || op == 5 || op == 6) ? fmin(x, y) : fmax(x, y));
}
__device__ inline double red_identity(int op) {
  return (op == 0 || op == 3) ? 0.0
                              : ((op == 2 || op == 5 || op == 6) ? INFINITY : (op == 4 ? -INFINITY : 0.0));
}

struct RedArgs {
  int op;
  long long n;
  const double* a; const double* b; const double* c; const double* d;
  double s1, s2;                        // step lengths (op 3)
  double* partial;                      // [RED_BLOCKS]
  double* out;                          // device scalar
};

__device__ double block_reduce(int op, double v) {
  __shared__ double sh[RED_THREADS / 64];
  for (int off = 32; off > 0; off >>= 1) v = red_combine(op, v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = red_identity(op);
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) r = red_combine(op, r, sh[w]);
  __syncthreads();
  return r;
}

// One thread's share of a reduction: elements lo + threadIdx.x + k RED_THREADS
// below hi, combined in that order; the loads of four of them are issued
// before they are combined.
template <int OP, typename R>
__device__ __forceinline__ double red_term(const R& r, long long i, double s1, double s2) {
  switch (OP) {
    case 0: return r.a[i] * r.b[i];
    case 1: return fabs(r.a[i]);
    case 2: return (r.b[i] < 0.0) ? -r.a[i] / r.b[i] : INFINITY;
    case 3: return (r.a[i] + s1 * r.b[i]) * (r.c[i] + s2 * r.d[i]);
    case 4: return r.a[i] + r.b[i];
    case 6: return fmin((r.b[i] < 0.0) ? -r.a[i] / r.b[i] : INFINITY,
                        (r.d[i] < 0.0) ? -r.c[i] / r.d[i] : INFINITY);
    default: return r.a[i];
  }
}
template <int OP, typename R>
__device__ __forceinline__ double red_chunk_op(const R& r, long long lo, long long hi, double s1,
                                               double s2) {
  double v = red_identity(OP);
  long long i = lo + threadIdx.x;
  for (; i + 3 * RED_THREADS < hi; i += 4 * RED_THREADS) {
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = red_term<OP>(r, i + u * RED_THREADS, s1, s2);
#pragma unroll
    for (int u = 0; u < 4; ++u) v = red_combine(OP, v, t[u]);
  }
  for (; i < hi; i += RED_THREADS) v = red_combine(OP, v, red_term<OP>(r, i, s1, s2));
  return v;
}
template <typename R>
__device__ double red_chunk(const R& r, long long lo, long long hi, double s1, double s2) {
  switch (r.op) {
    case 0: return red_chunk_op<0>(r, lo, hi, s1, s2);
    case 1: return red_chunk_op<1>(r, lo, hi, s1, s2);
    case 2: return red_chunk_op<2>(r, lo, hi, s1, s2);
    case 3: return red_chunk_op<3>(r, lo, hi, s1, s2);
    case 4: return red_chunk_op<4>(r, lo, hi, s1, s2);
    case 6: return red_chunk_op<6>(r, lo, hi, s1, s2);
    default: return red_chunk_op<5>(r, lo, hi, s1, s2);
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce1(RedArgs r) {
  const long long chunk = (r.n + gridDim.x - 1) / gridDim.x;
  const long long lo = blockIdx.x * chunk;
  const long long hi = lo + chunk < r.n ? lo + chunk : r.n;
  const double s1 = r.s1, s2 = r.s2;
  double v = red_chunk(r, lo, hi, s1, s2);
  v = block_reduce(r.op, v);
  if (threadIdx.x == 0) r.partial[blockIdx.x] = v;
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce2(RedArgs r, int nparts) {
  double v = red_identity(r.op);
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v = red_combine(r.op, v, r.partial[i]);
  v = block_reduce(r.op, v);
  if (threadIdx.x == 0) *r.out = v;
}

// Several independent reductions in one pair of launches: blockIdx.y selects
// the reduction; the per-reduction work split and trees are the same fixed
// ones as k_reduce1/k_reduce2, so results do not depend on how many share a
// launch.
__global__ __launch_bounds__(RED_THREADS) void k_mreduce1(MultiRed m) {
  const RedSpec& r = m.r[blockIdx.y];
  const long long chunk = (r.n + gridDim.x - 1) / gridDim.x;
  const long long lo = blockIdx.x * chunk;
  const long long hi = lo + chunk < r.n ? lo + chunk : r.n;
  const double s1 = r.ps1 ? fmin(1.0, *r.ps1) : r.s1;
  const double s2 = r.ps2 ? fmin(1.0, *r.ps2) : r.s2;
  double v = red_chunk(r, lo, hi, s1, s2);
  v = block_reduce(r.op, v);
  if (threadIdx.x == 0) m.partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = v;
}

__global__ __launch_bounds__(RED_THREADS) void k_mreduce2(MultiRed m, int nparts) {
  const RedSpec& r = m.r[blockIdx.x];
  double v = red_identity(r.op);
  for (int i = threadIdx.x; i < nparts; i += blockDim.x)
    v = red_combine(r.op, v, m.partial[(long long)blockIdx.x * nparts + i]);
  v = block_reduce(r.op, v);
  if (threadIdx.x == 0) m.out[r.slot] = v;
}

// ------------------------------------------------------------ launchers
void launch_mreduce(hipStream_t st, const MultiRed& m) {
  if (m.nred <= 0) return;
  hipLaunchKernelGGL(k_mreduce1, dim3(RED_BLOCKS, m.nred), dim3(RED_THREADS), 0, st, m);
  hipLaunchKernelGGL(k_mreduce2, dim3(m.nred), dim3(RED_THREADS), 0, st, m, RED_BLOCKS);
}

static inline int grid1d(long long n) {
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_pad_x(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                  long long d0off, const double* x, double* xp, const double* scale) {
  hipLaunchKernelGGL(k_pad_x, dim3(N + 1), dim3(256), 0, st, blk, N, n0, x0off, d0off, x, xp, scale);
}
void launch_wscaled(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                    long long d0off, const double* a, const double* b, const double* xs,
                    const double* Dp, double* w) {
  hipLaunchKernelGGL(k_wscaled, dim3(N + 1), dim3(256), 0, st, blk, N, n0, x0off, d0off, a, b, xs,
                     Dp, w);
}
void launch_combine(hipStream_t st, long long n, const double* t, double smu, const double* a,
                    const double* b, double* out, const double* smu_dev) {
  hipLaunchKernelGGL(k_combine, dim3(grid1d(n)), dim3(256), 0, st, n, t, smu, smu_dev, a, b, out);
}
void launch_sigma_mu(hipStream_t st, double* scal, long long n, int s_xz, int s_muaff, int s_out,
                     int s_sw, int s_muaff_sw) {
  hipLaunchKernelGGL(k_sigma_mu, dim3(1), dim3(64), 0, st, scal, 1.0 / (double)n, s_xz, s_muaff, s_out,
                     s_sw, s_muaff_sw);
}
void launch_bnd_prep(hipStream_t st, long long n, const double* ub, const double* x,
                     const double* z, const double* s, const double* w, double* ru, double* q,
                     double* zw, DevInfo* info) {
  hipLaunchKernelGGL(k_bnd_prep, dim3(grid1d(n)), dim3(256), 0, st, n, ub, x, z, s, w, ru, q, zw, info);
}
void launch_bnd_start(hipStream_t st, long long n, const double* ub, const double* x, double* z,
                      double* s, double* w, double* sm, double* wm) {
  hipLaunchKernelGGL(k_bnd_start, dim3(grid1d(n)), dim3(256), 0, st, n, ub, x, z, s, w, sm, wm);
}
void launch_bnd_shift(hipStream_t st, long long n, const double* ub, double a, double c,
                      double* x, double* z, double* s, double* w, double* sm, double* wm) {
  hipLaunchKernelGGL(k_bnd_shift, dim3(grid1d(n)), dim3(256), 0, st, n, ub, a, c, x, z, s, w, sm, wm);
}
void launch_gondzio_rhs(hipStream_t st, long long n, const double* x, const double* z,
                        const double* dx, const double* dz, double at_p, double at_d,
                        const double* smu, double beta_min, double beta_max, double* r) {
  if (n > 0)
    hipLaunchKernelGGL(k_gondzio_rhs, dim3(grid1d(n)), dim3(256), 0, st, n, x, z, dx, dz, at_p,
                       at_d, smu, beta_min, beta_max, r);
}
void launch_steps(hipStream_t st, double eta, const StepSet& s) {
  long long nmax = 0;
  for (int v = 0; v < s.cnt; ++v) nmax = s.n[v] > nmax ? s.n[v] : nmax;
  if (s.cnt > 0 && nmax > 0)
    hipLaunchKernelGGL(k_steps, dim3(grid1d(nmax), s.cnt), dim3(256), 0, st, s, eta);
}
void launch_pad_y(hipStream_t st, const BlockInfo* blk, int N, const double* y, double* yp) {
  hipLaunchKernelGGL(k_pad_y, dim3(N), dim3(256), 0, st, blk, y, yp);
}
void launch_rhx(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                long long d0off, const double* rx, const double* rz, const double* xs,
                const double* Dp, double* rhx, double* vx) {
  hipLaunchKernelGGL(k_rhx, dim3(N + 1), dim3(256), 0, st, blk, N, n0, x0off, d0off, rx, rz, xs,
                     Dp, rhx, vx);
}
void launch_rows_multi(hipStream_t st, const BlockInfo* blk, const int2* rowtiles, int nrt,
                       const double* A, const double* C, long long d0off, const RowsArgs& ra) {
  const dim3 g((nrt + 3) / 4), b(256);
  if (ra.nv == 1) hipLaunchKernelGGL(k_rows_nv<1>, g, b, 0, st, blk, rowtiles, nrt, A, C, d0off, ra);
  else if (ra.nv == 2) hipLaunchKernelGGL(k_rows_nv<2>, g, b, 0, st, blk, rowtiles, nrt, A, C, d0off, ra);
  else hipLaunchKernelGGL(k_rows_nv<3>, g, b, 0, st, blk, rowtiles, nrt, A, C, d0off, ra);
}
void launch_rows(hipStream_t st, const BlockInfo* blk, const int2* rowtiles, int nrt,
                 const double* A, const double* C, const double* xp, long long d0off,
                 const double* base, double alpha, int with_C, int padded_out, double* out) {
  RowsArgs ra{};
  ra.nv = 1;
  ra.v[0] = xp; ra.base[0] = base; ra.alpha[0] = alpha; ra.out[0] = out;
  ra.with_C[0] = with_C; ra.padded[0] = padded_out; ra.chain[0] = 0;
  launch_rows_multi(st, blk, rowtiles, nrt, A, C, d0off, ra);
}
void launch_linkrows(hipStream_t st, const BlockInfo* blk, int P, int ng, int n0,
                     const int* lsz, const long long* loff, long long nl, const int* lptr,
                     const int* lcol, const double* lval, const int* gptr, const int* gidx,
                     const double* gval, const double* xp, const double* x0, const double* F0,
                     const double* F0L, const double* base, double alpha, double* out) {
  const int gridP = P > 0 ? (P < 1024 ? P : 1024) : 0;
  if (gridP + ng <= 0) return;
  hipLaunchKernelGGL(k_linkrows, dim3(gridP + ng), dim3(256), 0, st, blk, P, gridP, n0, lsz, loff,
                     nl, lptr, lcol, lval, gptr, gidx, gval, xp, x0, F0, F0L, base, alpha, out);
}
void launch_cols(hipStream_t st, const BlockInfo* blk, const int2* coltiles, int nct,
                 const double* A, const double* yp, const double* yL, const int* cptr,
                 const int* crow, const double* cval, int mode, const double* cvec,
                 const double* zvec, const double* Dp, double* gout, double* out,
                 const DzArgs& dzv) {
  hipLaunchKernelGGL(k_cols, dim3((nct + 3) / 4), dim3(256), 0, st, blk, coltiles, nct, A, yp, yL,
                     cptr, crow, cval, mode, cvec, zvec, Dp, gout, out, dzv);
}
void launch_ccols(hipStream_t st, const BlockInfo* blk, const int2* ctiles, int nctile, int n0,
                  const double* C, const double* yp, double* part) {
  if (nctile > 0 && n0 > 0)
    hipLaunchKernelGGL(k_ccols, dim3((nctile + 3) / 4), dim3(256), 0, st, blk, ctiles, nctile, n0,
                       C, yp, part);
}
void launch_x0_sum(hipStream_t st, int N, int n0, long long nl, long long f0first,
                   const double* part, const double* F0, const double* yL, int mode,
                   const double* cvec, const double* zvec, long long x0off, double* gout,
                   double* out) {
  if (n0 > 0)
    hipLaunchKernelGGL(k_x0_sum, dim3(n0), dim3(256), 0, st, N, n0, nl, f0first, part, F0, yL, mode,
                       cvec, zvec, x0off, gout, out);
}
template <typename T>
void launch_block_fwd(hipStream_t st, const BlockInfo* blk, int N, int max_rt, const T* LB,
                      const T* LINV, const double* tin, double* tv, double* qn) {
  const size_t sh = (size_t)TS * max_rt * sizeof(double);
  hipLaunchKernelGGL(k_block_fwd<T>, dim3(N), dim3(256), sh, st, blk, LB, LINV, tin, tv, qn);
}
template <typename T>
void launch_block_bwd(hipStream_t st, const BlockInfo* blk, int N, int nb, long long nl,
                      int max_rt, const T* LB, const T* LINV, const double* v, const double* u,
                      double* dy, double* dyp) {
  const size_t sh = (size_t)TS * max_rt * sizeof(double);
  hipLaunchKernelGGL(k_block_bwd<T>, dim3(N), dim3(256), sh, st, blk, nb, nl, LB, LINV, v, u, dy,
                     dyp);
}
template void launch_block_fwd<double>(hipStream_t, const BlockInfo*, int, int, const double*,
                                       const double*, const double*, double*, double*);
template void launch_block_fwd<float>(hipStream_t, const BlockInfo*, int, int, const float*,
                                      const float*, const double*, double*, double*);
template void launch_block_bwd<double>(hipStream_t, const BlockInfo*, int, int, long long, int,
                                       const double*, const double*, const double*,
                                       const double*, double*, double*);
template void launch_block_bwd<float>(hipStream_t, const BlockInfo*, int, int, long long, int,
                                      const float*, const float*, const double*, const double*,
                                      double*, double*);
void launch_schur_rhs(hipStream_t st, const BlockInfo* blk, int N, int nb, const int* lsz,
                      const long long* loff, long long nl, const double* qn, const double* rhx0,
                      double* s) {
  const int P = N - 1;
  const int npb = P > 0 ? (P < 1024 ? P : 1024) : 0;
  if (npb + nb > 0)
    hipLaunchKernelGGL(k_schur_rhs, dim3(npb + nb), dim3(256), 0, st, blk, N, nb, lsz, loff, nl,
                       npb, qn, rhx0, s);
}
void launch_solve_tail(hipStream_t st, int N, int n0, long long nl, long long f0first,
                       const double* part, const double* F0, const double* u, long long x0off,
                       long long mblk, double* gout, double* dx, const DzArgs& dzv, double* dy) {
  long long nb = (nl + 255) / 256;
  if (nb > 64) nb = 64;
  const int grid = n0 + (int)nb;
  if (grid > 0)
    hipLaunchKernelGGL(k_solve_tail, dim3(grid), dim3(256), 0, st, N, n0, nl, f0first, part, F0, u,
                       x0off, mblk, gout, dx, dzv, dy);
}
void launch_check_prep(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                       long long d0off, const double* rx, const double* rz, const double* g,
                       const double* dx, const double* dz, const double* xs, const double* zs,
                       const double* Dp, double* ex, double* ez, double* xp, double* w2p,
                       const BndArgs& b) {
  hipLaunchKernelGGL(k_check_prep, dim3(N + 1), dim3(256), 0, st, blk, N, n0, x0off, d0off, rx, rz,
                     g, dx, dz, xs, zs, Dp, ex, ez, xp, w2p, b);
}
void launch_resid_prep(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                       long long d0off, const double* x, const double* z, const double* rd,
                       const double* xs, const double* Dp, double* rzv, double* rhx, double* vx,
                       double* w1p, double* xp, const BndArgs& b, double* rdt_out) {
  hipLaunchKernelGGL(k_resid_prep, dim3(N + 1), dim3(256), 0, st, blk, N, n0, x0off, d0off, x, z,
                     rd, xs, Dp, rzv, rhx, vx, w1p, xp, b, rdt_out);
}
void launch_adj_scale(hipStream_t st, long long n, int mode, const double* zs, const double* v,
                      double* out) {
  if (n > 0) hipLaunchKernelGGL(k_adj_scale, dim3(grid1d(n)), dim3(256), 0, st, n, mode, zs, v, out);
}
void launch_axpy(hipStream_t st, long long n, double a, const double* x, double* y) {
  if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(grid1d(n)), dim3(256), 0, st, n, a, x, y);
}
void launch_dz(hipStream_t st, long long n, const double* rz, const double* zs, const double* xs,
               const double* dx, double* dz) {
  hipLaunchKernelGGL(k_dz, dim3(grid1d(n)), dim3(256), 0, st, n, rz, zs, xs, dx, dz);
}
void launch_rd(hipStream_t st, long long n, const double* c, const double* g, const double* z,
               double* rd) {
  hipLaunchKernelGGL(k_rd, dim3(grid1d(n)), dim3(256), 0, st, n, c, g, z, rd);
}
void launch_res_x(hipStream_t st, long long n, const double* rx, const double* rz,
                  const double* g, const double* dx, const double* dz, const double* xs,
                  const double* zs, double* ex, double* ez) {
  hipLaunchKernelGGL(k_res_x, dim3(grid1d(n)), dim3(256), 0, st, n, rx, rz, g, dx, dz, xs, zs, ex,
                     ez);
}
void launch_copy(hipStream_t st, long long n, const double* src, double* dst) {
  if (n > 0) hipLaunchKernelGGL(k_copy, dim3(grid1d(n)), dim3(256), 0, st, n, src, dst);
}
void launch_rz(hipStream_t st, long long n, int mode, const double* x, const double* z,
               const double* dxa, const double* dza, double smu, double* rz, const double* smu_dev,
               const BndArgs* b, double* rxc) {
  BndArgs nb{};
  hipLaunchKernelGGL(k_rz, dim3(grid1d(n)), dim3(256), 0, st, n, mode, x, z, dxa, dza, smu, smu_dev,
                     rz, b ? *b : nb, b ? rxc : nullptr);
}
void launch_fill(hipStream_t st, long long n, double v, double* dst) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(256), 0, st, n, v, dst);
}
void launch_addscalar(hipStream_t st, long long n, double v, double* dst) {
  if (n > 0) hipLaunchKernelGGL(k_addscalar, dim3(grid1d(n)), dim3(256), 0, st, n, v, dst);
}
void launch_reduce(hipStream_t st, int op, long long n, const double* a, const double* b,
                   const double* c, const double* d, double s1, double s2,
                   double* partial, double* out) {
  RedArgs r{op, n, a, b, c, d, s1, s2, partial, out};
  hipLaunchKernelGGL(k_reduce1, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, r);
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(RED_THREADS), 0, st, r, RED_BLOCKS);
}

}  // namespace ahlp
