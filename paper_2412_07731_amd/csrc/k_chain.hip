// Factorization and solve of the Schur complement (a6)
//
//     S = [ T   E  ]     T: block tridiagonal over the P = N-1 link pairs
//         [ E'  S00]     E: link pairs x linking variables, S00: x_0 block
//
// T is positive definite and the border Schur complement S00 - E'T^-1 E
// negative definite, so S = L diag(I, -I) L' with two Choleskys.  A plain
// block Cholesky of T is a chain of P dependent steps.  Following the
// splitting of the link chain into consecutive subsets of Sec. 4.2 (there used
// to distribute the chain over process groups), the pairs are cut into G
// segments separated by single separator pairs:
//
//   level 1  every segment eliminates its interior pairs in order, in parallel
//            with the others (one workgroup per segment).  Its first pair is
//            coupled to the left separator, whose coupling moves along the
//            segment as fill; its last pair is coupled to the right separator.
//            Each segment leaves updates for the two separators, a coupling
//            between them and an update of S00.
//   level 2  the separators form again a block-tridiagonal chain with the same
//            border; one workgroup eliminates it and factors the border.
//
// The dependency depth is about P/G + G instead of P.  Every reduction is done
// by one thread in a fixed order, so results are reproducible run to run.
// Matrices are column-major; pair j has size l_j.
#include "common.h"
#include "kernels.h"
#include "small_dense.h"

namespace ahlp {

// ------------------------------------------------------- level 1 factor
__global__ void k_chain_seg_factor(ChainArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  const int L2 = c.lmax * c.lmax, n0 = c.n0;
  double* cur = sm;
  double* Li = cur + L2;
  double* Yn = Li + L2;
  double* Z = Yn + L2;
  double* ZF = Z + L2;
  double* Ec = ZF + L2;
  double* Gk = Ec + c.lmax * n0;

  const int g = blockIdx.x;
  const int a = c.seg[g].x, b = c.seg[g].y;
  const bool hasL = g > 0, hasR = g < c.G - 1;
  const int sL = a - 1, sR = b;
  const int lsL = hasL ? c.l[sL] : 0, lsR = hasR ? c.l[sR] : 0;
  double* slot = c.segout + (long long)g * SEG_STRIDE;
  double* dDiagL = so_diagL(slot);
  double* dEL = so_EL(slot);
  double* dS00 = so_S00(slot);
  for (int i = threadIdx.x; i < lsL * lsL; i += blockDim.x) dDiagL[i] = 0.0;
  for (int i = threadIdx.x; i < lsL * n0; i += blockDim.x) dEL[i] = 0.0;
  for (int i = threadIdx.x; i < n0 * n0; i += blockDim.x) dS00[i] = 0.0;

  int la = c.l[a];
  sm_copy(cur, c.Td + c.tdoff[a], la * la);
  sm_copy(Ec, c.E + c.eoff[a], la * n0);
  if (hasL) {  // coupling of the left separator with pair a: T[a-1, a] = T[a, a-1]'
    const double* Ta = c.To + c.tooff[a - 1];  // l_a x l_{a-1}
    for (int idx = threadIdx.x; idx < lsL * la; idx += blockDim.x) {
      const int i = idx % lsL, j = idx / lsL;
      ZF[i + j * lsL] = Ta[j + i * la];
    }
    __syncthreads();
  }
  int cnt = 0;
  for (int k = a; k < b; ++k) {
    const int lk = c.l[k];
    cnt += sm_chol(cur, lk, c.thrT[k]);
    sm_trinv(cur, Li, lk);
    for (int i = threadIdx.x; i < lk * lk; i += blockDim.x) {
      c.CL[c.tdoff[k] + i] = cur[i];
      c.CLi[c.tdoff[k] + i] = Li[i];
    }
    const int nxt = (k + 1 < b) ? k + 1 : (hasR ? sR : -1);
    const int ln = nxt >= 0 ? c.l[nxt] : 0;
    // Yn = T[nxt,k] L^-T,  Z = T[sL,k] L^-T,  G = L^-1 E_k
    if (ln > 0) sm_gemm(Yn, ln, nullptr, 0, 0.0, c.To + c.tooff[k], ln, false, Li, lk, true, ln, lk, lk, 1.0);
    if (lsL > 0) sm_gemm(Z, lsL, nullptr, 0, 0.0, ZF, lsL, false, Li, lk, true, lsL, lk, lk, 1.0);
    if (n0 > 0) sm_gemm(Gk, lk, nullptr, 0, 0.0, Li, lk, false, Ec, lk, false, lk, n0, lk, 1.0);
    for (int i = threadIdx.x; i < ln * lk; i += blockDim.x) c.CYn[c.tooff[k] + i] = Yn[i];
    for (int i = threadIdx.x; i < lsL * lk; i += blockDim.x) c.CZ[c.zoff[k] + i] = Z[i];
    for (int i = threadIdx.x; i < lk * n0; i += blockDim.x) c.CG[c.eoff[k] + i] = Gk[i];
    // updates of the left separator and of the border
    if (lsL > 0) {
      sm_gemm(dDiagL, lsL, dDiagL, lsL, 1.0, Z, lsL, false, Z, lsL, true, lsL, lsL, lk, -1.0);
      if (n0 > 0) sm_gemm(dEL, lsL, dEL, lsL, 1.0, Z, lsL, false, Gk, lk, false, lsL, n0, lk, -1.0);
    }
    if (n0 > 0) sm_gemm(dS00, n0, dS00, n0, 1.0, Gk, lk, true, Gk, lk, false, n0, n0, lk, -1.0);
    if (k + 1 < b) {
      const int l1 = ln;
      sm_gemm(cur, l1, c.Td + c.tdoff[k + 1], l1, 1.0, Yn, l1, false, Yn, l1, true, l1, l1, lk, -1.0);
      if (n0 > 0) sm_gemm(Ec, l1, c.E + c.eoff[k + 1], l1, 1.0, Yn, l1, false, Gk, lk, false, l1, n0, lk, -1.0);
      if (lsL > 0) sm_gemm(ZF, lsL, nullptr, 0, 0.0, Z, lsL, false, Yn, l1, true, lsL, l1, lk, -1.0);
    } else if (hasR) {
      sm_gemm(so_diagR(slot), lsR, nullptr, 0, 0.0, Yn, lsR, false, Yn, lsR, true, lsR, lsR, lk, -1.0);
      if (n0 > 0) sm_gemm(so_ER(slot), lsR, nullptr, 0, 0.0, Yn, lsR, false, Gk, lk, false, lsR, n0, lk, -1.0);
      if (lsL > 0) sm_gemm(so_off(slot), lsR, nullptr, 0, 0.0, Yn, lsR, false, Z, lsL, true, lsR, lsL, lk, -1.0);
    }
  }
  if (threadIdx.x == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// ------------------------------------------------------- level 2 factor
__global__ void k_chain_sep_factor(ChainArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  const int L2 = c.lmax * c.lmax, n0 = c.n0;
  double* cur = sm;
  double* Li = cur + L2;
  double* Y = Li + L2;
  double* Ec = Y + L2;
  double* Gs = Ec + c.lmax * n0;
  const int S = c.G - 1;
  double* S00w = c.S00w;
  // S00' = S00 + sum over segments (fixed order)
  for (int idx = threadIdx.x; idx < n0 * n0; idx += blockDim.x) {
    double v = c.S00[idx];
    for (int g = 0; g < c.G; ++g) v += so_S00(c.segout + (long long)g * SEG_STRIDE)[idx];
    S00w[idx] = v;
  }
  __syncthreads();
  int cnt = 0;
  for (int s = 0; s < S; ++s) {
    const int p = c.seg[s].y;
    const int lp = c.l[p];
    double* sl = c.segout + (long long)s * SEG_STRIDE;        // segment s: this is its right sep
    double* sr = c.segout + (long long)(s + 1) * SEG_STRIDE;  // segment s+1: this is its left sep
    // reduced diagonal and border rows of separator s (minus the previous step's update)
    for (int idx = threadIdx.x; idx < lp * lp; idx += blockDim.x) {
      double v = c.Td[c.tdoff[p] + idx] + so_diagR(sl)[idx] + so_diagL(sr)[idx];
      if (s > 0) {
        const int i = idx % lp, j = idx / lp;
        const int lq = c.l[c.seg[s - 1].y];
        double u = 0.0;
        for (int k = 0; k < lq; ++k) u += Y[i + k * lp] * Y[j + k * lp];
        v -= u;
      }
      cur[idx] = v;
    }
    for (int idx = threadIdx.x; idx < lp * n0; idx += blockDim.x) {
      double v = c.E[c.eoff[p] + idx] + so_ER(sl)[idx] + so_EL(sr)[idx];
      if (s > 0) {
        const int i = idx % lp, j = idx / lp;
        const int lq = c.l[c.seg[s - 1].y];
        double u = 0.0;
        for (int k = 0; k < lq; ++k) u += Y[i + k * lp] * Gs[k + j * lq];
        v -= u;
      }
      Ec[idx] = v;
    }
    __syncthreads();
    cnt += sm_chol(cur, lp, c.thrT[p]);
    sm_trinv(cur, Li, lp);
    for (int i = threadIdx.x; i < lp * lp; i += blockDim.x) {
      c.CL[c.tdoff[p] + i] = cur[i];
      c.CLi[c.tdoff[p] + i] = Li[i];
    }
    if (n0 > 0) {
      sm_gemm(Gs, lp, nullptr, 0, 0.0, Li, lp, false, Ec, lp, false, lp, n0, lp, 1.0);
      for (int i = threadIdx.x; i < lp * n0; i += blockDim.x) c.CG[c.eoff[p] + i] = Gs[i];
      sm_gemm(S00w, n0, S00w, n0, 1.0, Gs, lp, true, Gs, lp, false, n0, n0, lp, -1.0);
    }
    if (s + 1 < S) {
      // coupling of separator s+1 with separator s comes from segment s+1
      const int lq = c.l[c.seg[s + 1].y];
      sm_gemm(Y, lq, nullptr, 0, 0.0, so_off(sr), lq, false, Li, lp, true, lq, lp, lp, 1.0);
      for (int i = threadIdx.x; i < lq * lp; i += blockDim.x) c.CSub[c.suboff[s + 1] + i] = Y[i];
      __syncthreads();
    }
  }
  // border (global rows, then x_0): -(S00') = Lb T Lb' with T = diag(-I, I)
  // (the global rows' part is positive definite in S00', x_0's negative
  // definite), Lbi = Lb^-1
  if (n0 > 0) {
    double* B = sm;
    double* Bi = sm + n0 * n0;
    __shared__ double s_max;
    for (int idx = threadIdx.x; idx < n0 * n0; idx += blockDim.x) B[idx] = -S00w[idx];
    __syncthreads();
    if (threadIdx.x == 0) {
      double md = 0.0;
      for (int i = 0; i < n0; ++i) md = fmax(md, fabs(B[i + i * n0]));
      s_max = md;
    }
    __syncthreads();
    cnt += sm_chol_signed(B, n0, c.ng, PIVOT_REL * s_max);
    sm_trinv(B, Bi, n0);
    for (int i = threadIdx.x; i < n0 * n0; i += blockDim.x) {
      c.Lb[i] = B[i];
      c.Lbi[i] = Bi[i];
    }
  }
  if (threadIdx.x == 0 && cnt) atomicAdd(&c.info->pivots, cnt);
}

// ------------------------------------------------------- solve
__global__ void k_chain_seg_fwd(ChainSolveArgs a) {
  const ChainArgs& c = a.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* r = reinterpret_cast<double*>(smem_raw);
  const int g = blockIdx.x, n0 = c.n0;
  const int ka = c.seg[g].x, kb = c.seg[g].y;
  const bool hasL = g > 0, hasR = g < c.G - 1;
  const int lsL = hasL ? c.l[ka - 1] : 0, lsR = hasR ? c.l[kb] : 0;
  double* out = a.segrhs + (long long)g * SEGRHS_STRIDE;
  double* dsL = out;
  double* dsR = out + LMAX;
  double* ds0 = out + 2 * LMAX;
  for (int i = threadIdx.x; i < lsL; i += blockDim.x) dsL[i] = 0.0;
  for (int i = threadIdx.x; i < n0; i += blockDim.x) ds0[i] = 0.0;
  __syncthreads();
  for (int k = ka; k < kb; ++k) {
    const int lk = c.l[k];
    const double* sk = a.s + a.loff[k];
    if (k > ka) {
      const int lp = c.l[k - 1];
      sm_gemv(r, sk, c.CYn + c.tooff[k - 1], lk, false, a.w + a.loff[k - 1], lk, lp, -1.0);
    } else {
      sm_copy(r, sk, lk);
    }
    double* wk = a.w + a.loff[k];
    sm_gemv(wk, nullptr, c.CLi + c.tdoff[k], lk, false, r, lk, lk, 1.0);
    if (lsL > 0) sm_gemv(dsL, dsL, c.CZ + c.zoff[k], lsL, false, wk, lsL, lk, -1.0);
    if (n0 > 0) sm_gemv(ds0, ds0, c.CG + c.eoff[k], lk, true, wk, n0, lk, -1.0);
  }
  if (hasR) sm_gemv(dsR, nullptr, c.CYn + c.tooff[kb - 1], lsR, false, a.w + a.loff[kb - 1], lsR, c.l[kb - 1], -1.0);
}

__global__ void k_chain_sep_solve(ChainSolveArgs a) {
  const ChainArgs& c = a.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* r = reinterpret_cast<double*>(smem_raw);
  double* s0 = r + LMAX;
  double* w0 = s0 + N0MAX;
  const int n0 = c.n0, S = c.G - 1;
  for (int i = threadIdx.x; i < n0; i += blockDim.x) {
    double v = a.s[a.nl + i];
    for (int g = 0; g < c.G; ++g) v += (a.segrhs + (long long)g * SEGRHS_STRIDE + 2 * LMAX)[i];
    s0[i] = v;
  }
  __syncthreads();
  for (int sidx = 0; sidx < S; ++sidx) {
    const int p = c.seg[sidx].y, lp = c.l[p];
    const double* dR = a.segrhs + (long long)sidx * SEGRHS_STRIDE + LMAX;   // segment s (right sep)
    const double* dL = a.segrhs + (long long)(sidx + 1) * SEGRHS_STRIDE;    // segment s+1 (left sep)
    for (int i = threadIdx.x; i < lp; i += blockDim.x) r[i] = a.s[a.loff[p] + i] + dR[i] + dL[i];
    __syncthreads();
    if (sidx > 0) {
      const int q = c.seg[sidx - 1].y;
      sm_gemv(r, r, c.CSub + c.suboff[sidx], lp, false, a.w + a.loff[q], lp, c.l[q], -1.0);
    }
    double* wp = a.w + a.loff[p];
    sm_gemv(wp, nullptr, c.CLi + c.tdoff[p], lp, false, r, lp, lp, 1.0);
    if (n0 > 0) sm_gemv(s0, s0, c.CG + c.eoff[p], lp, true, wp, n0, lp, -1.0);
  }
  double* u0 = a.u + a.nl;
  if (n0 > 0) {
    // S00' u0 = s0 with -(S00') = Lb T Lb':  u0 = -Lb^-T T Lb^-1 s0
    sm_gemv(w0, nullptr, c.Lbi, n0, false, s0, n0, n0, 1.0);
    for (int i = threadIdx.x; i < c.ng; i += blockDim.x) w0[i] = -w0[i];
    __syncthreads();
    sm_gemv(u0, nullptr, c.Lbi, n0, true, w0, n0, n0, -1.0);
  }
  for (int sidx = S - 1; sidx >= 0; --sidx) {
    const int p = c.seg[sidx].y, lp = c.l[p];
    for (int i = threadIdx.x; i < lp; i += blockDim.x) r[i] = a.w[a.loff[p] + i];
    __syncthreads();
    if (sidx + 1 < S) {
      const int q = c.seg[sidx + 1].y;
      sm_gemv(r, r, c.CSub + c.suboff[sidx + 1], c.l[q], true, a.u + a.loff[q], lp, c.l[q], -1.0);
    }
    if (n0 > 0) sm_gemv(r, r, c.CG + c.eoff[p], lp, false, u0, lp, n0, -1.0);
    sm_gemv(a.u + a.loff[p], nullptr, c.CLi + c.tdoff[p], lp, true, r, lp, lp, 1.0);
  }
}

__global__ void k_chain_seg_bwd(ChainSolveArgs a) {
  const ChainArgs& c = a.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* r = reinterpret_cast<double*>(smem_raw);
  const int g = blockIdx.x, n0 = c.n0;
  const int ka = c.seg[g].x, kb = c.seg[g].y;
  const bool hasL = g > 0, hasR = g < c.G - 1;
  const int lsL = hasL ? c.l[ka - 1] : 0;
  const double* u0 = a.u + a.nl;
  for (int k = kb - 1; k >= ka; --k) {
    const int lk = c.l[k];
    sm_copy(r, a.w + a.loff[k], lk);
    const int nxt = (k + 1 < kb) ? k + 1 : (hasR ? kb : -1);
    if (nxt >= 0)
      sm_gemv(r, r, c.CYn + c.tooff[k], c.l[nxt], true, a.u + a.loff[nxt], lk, c.l[nxt], -1.0);
    if (lsL > 0) sm_gemv(r, r, c.CZ + c.zoff[k], lsL, true, a.u + a.loff[ka - 1], lk, lsL, -1.0);
    if (n0 > 0) sm_gemv(r, r, c.CG + c.eoff[k], lk, false, u0, lk, n0, -1.0);
    sm_gemv(a.u + a.loff[k], nullptr, c.CLi + c.tdoff[k], lk, true, r, lk, lk, 1.0);
  }
}

// ------------------------------------------------------------- launchers
size_t chain_factor_smem(int lmax, int n0) {
  size_t a = (size_t)(5 * lmax * lmax + 2 * lmax * n0) * sizeof(double);
  size_t b = (size_t)(3 * lmax * lmax + 2 * lmax * n0) * sizeof(double);
  size_t c = (size_t)(2 * n0 * n0) * sizeof(double);
  size_t m = a > b ? a : b;
  return m > c ? m : c;
}

void launch_chain_factor(hipStream_t st, const ChainArgs& c) {
  const size_t sh = chain_factor_smem(c.lmax, c.n0);
  if (c.G > 0) hipLaunchKernelGGL(k_chain_seg_factor, dim3(c.G), dim3(64), sh, st, c);
  hipLaunchKernelGGL(k_chain_sep_factor, dim3(1), dim3(256), sh, st, c);
}

void launch_chain_solve(hipStream_t st, const ChainSolveArgs& a) {
  const size_t sh = (size_t)(LMAX + 2 * N0MAX) * sizeof(double);
  if (a.c.G > 0) hipLaunchKernelGGL(k_chain_seg_fwd, dim3(a.c.G), dim3(64), sh, st, a);
  hipLaunchKernelGGL(k_chain_sep_solve, dim3(1), dim3(64), sh, st, a);
  if (a.c.G > 0) hipLaunchKernelGGL(k_chain_seg_bwd, dim3(a.c.G), dim3(64), sh, st, a);
}

void set_chain_smem_limits(size_t bytes) {
  hipFuncSetAttribute((const void*)k_chain_seg_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  hipFuncSetAttribute((const void*)k_chain_sep_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace ahlp
