// Small dense kernels-within-kernels for the Schur-complement chain: every
// thread of the workgroup takes part and each routine ends with a barrier.
// Matrices are column-major.
#pragma once

#include "common.h"

namespace ahlp {

// ---------------------------------------------------------- small helpers
// All threads of the workgroup take part; each ends with a barrier.

// C = (Cs ? beta*Cs : 0) + alpha * opA(A) * opB(B);  C: M x N (ldc), K inner.
// opA(A)[i,k] = ta ? A[k + i*lda] : A[i + k*lda]; opB(B)[k,j] = tb ? B[j + k*ldb] : B[k + j*ldb].
__device__ inline void sm_gemm(double* C, int ldc, const double* Cs, int ldcs, double beta,
                        const double* A, int lda, bool ta, const double* B, int ldb, bool tb,
                        int M, int N, int K, double alpha) {
  for (int idx = threadIdx.x; idx < M * N; idx += blockDim.x) {
    const int i = idx % M, j = idx / M;
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
      const double a = ta ? A[k + i * lda] : A[i + k * lda];
      const double b = tb ? B[j + k * ldb] : B[k + j * ldb];
      s += a * b;
    }
    double v = alpha * s;
    if (Cs) v += beta * Cs[i + j * ldcs];
    C[i + j * ldc] = v;
  }
  __syncthreads();
}

// y = (ys ? ys : 0) + alpha * op(A) x;  op(A): M x K.
__device__ inline void sm_gemv(double* y, const double* ys, const double* A, int lda, bool ta,
                        const double* x, int M, int K, double alpha) {
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += (ta ? A[k + i * lda] : A[i + k * lda]) * x[k];
    y[i] = (ys ? ys[i] : 0.0) + alpha * s;
  }
  __syncthreads();
}

__device__ inline void sm_copy(double* dst, const double* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

// In-place lower Cholesky with the pivot rule (upper part zeroed).  Returns the
// number of replaced pivots (same value in every thread).
__device__ inline int sm_chol(double* A, int n, double thr) {
  __shared__ double s_l;
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double d = A[j + j * n];
      if (!(d > thr)) {
        d = PIVOT_BIG;
        ++s_cnt;
      }
      s_l = sqrt(d);
      A[j + j * n] = s_l;
    }
    __syncthreads();
    const double ljj = s_l;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[i + j * n] /= ljj;
    __syncthreads();
    const int r = n - j - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
      const int i = j + 1 + idx % r, k = j + 1 + idx / r;
      if (i >= k) A[i + k * n] -= A[i + j * n] * A[k + j * n];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, k = idx / n;
    if (i < k) A[idx] = 0.0;
  }
  __syncthreads();
  return s_cnt;
}

// Signed lower Cholesky of a quasi-definite matrix, in place: A = L T L' with
// T = diag(-1 for the first nneg columns, +1 after) and L with a positive
// diagonal (the pivot of column j is T_jj times the updated diagonal; the
// pivot rule applies to it).  nneg = 0 is sm_chol.  Returns the number of
// replaced pivots (same value in every thread).
__device__ inline int sm_chol_signed(double* A, int n, int nneg, double thr) {
  __shared__ double s_l;
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  for (int j = 0; j < n; ++j) {
    const double tj = j < nneg ? -1.0 : 1.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      double d = tj * A[j + j * n];
      if (!(d > thr)) {
        d = PIVOT_BIG;
        ++s_cnt;
      }
      s_l = sqrt(d);
      A[j + j * n] = s_l;
    }
    __syncthreads();
    const double ljj = s_l;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[i + j * n] = tj * A[i + j * n] / ljj;
    __syncthreads();
    const int r = n - j - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
      const int i = j + 1 + idx % r, k = j + 1 + idx / r;
      if (i >= k) A[i + k * n] -= tj * A[i + j * n] * A[k + j * n];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, k = idx / n;
    if (i < k) A[idx] = 0.0;
  }
  __syncthreads();
  return s_cnt;
}

// Li = L^-1 for lower triangular L (n x n); one thread per column.
__device__ inline void sm_trinv(const double* L, double* Li, int n) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      double s = (i == k) ? 1.0 : 0.0;
      for (int j = k; j < i; ++j) s -= L[i + j * n] * Li[j + k * n];
      Li[i + k * n] = (i >= k) ? s / L[i + i * n] : 0.0;
    }
  }
  __syncthreads();
}


}  // namespace ahlp
