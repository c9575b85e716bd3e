// Device ceilings for the measurement (not part of the method): the MFMA
// pipe's throughput on a dependency-free stream of the instructions the
// factorization kernels use (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32),
// the HBM read bandwidth of a streaming pass with the 16-byte nontemporal
// loads the row and column passes use, and the latency of the block
// factor's one-wave tile Cholesky, which sits on its dependency chain.  The
// kernels are reported against these beside the published peaks.
#include "common.h"
#include "kernels.h"
#include "tile_chol.h"

namespace ahlp {

namespace {

// Eight independent accumulators per wave, so the pipe always has an
// instruction whose inputs are ready; the operands depend on the lane so
// nothing folds, and the sums are written only if they take a value they
// cannot take, so nothing is removed.
template <typename T>
__global__ __launch_bounds__(256) void k_mfma_peak(int iters, double* __restrict__ out) {
  typedef typename Acc<T>::type AT;
  const int lane = threadIdx.x & 63;
  const T a = T(1) + T(lane) * T(1e-3), b = T(1) - T(lane & 7) * T(1e-3);
  AT acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = AT{0, 0, 0, 0};
  // sixteen rounds per loop trip, so the loop's own overhead (the compiler
  // moves the accumulators between register files at the back edge) is
  // amortized over 128 products
  for (int it = 0; it < iters; it += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] = mfma(a, b, acc[i]);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) s += (double)acc[i][k];
  if (s == -1.0) out[blockIdx.x] = s;
}

// Streaming read of n2 16-byte pairs: each thread a grid-strided share, four
// loads in flight, one partial sum per workgroup.
__global__ __launch_bounds__(256) void k_stream_read(const dv2* __restrict__ p, long long n2,
                                                     double* __restrict__ out) {
  const long long stride = (long long)gridDim.x * 256;
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const dv2 a = ld_stream2(p + i), b = ld_stream2(p + i + stride);
    const dv2 c = ld_stream2(p + i + 2 * stride), d = ld_stream2(p + i + 3 * stride);
    s0 += a.x + b.x + c.x + d.x;
    s1 += a.y + b.y + c.y + d.y;
  }
  for (; i < n2; i += stride) {
    const dv2 a = ld_stream2(p + i);
    s0 += a.x;
    s1 += a.y;
  }
  double s = s0 + s1;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// One wave factors the same well-conditioned padded LDS tile `iters` times
// with the panel factor's tile Cholesky (FP64).  With `beside`, four more
// waves stream FP64 MFMAs until it is done; with a workgroup's waves dealt
// round-robin to the SIMDs, the fifth shares the factoring wave's SIMD, as a
// co-resident block's wave does in the panel factor.  The streaming waves
// stop at the factoring wave's flag, or after a fixed number of trips.
__global__ __launch_bounds__(320) void k_chol_latency(int iters, double* __restrict__ out) {
  constexpr int LD = TS + 1, MAX_TRIPS = 1 << 17;
  __shared__ double P[TS * LD], Lt[TS * LD], Li[TS * LD];
  __shared__ int done;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < TS * LD; e += blockDim.x) {
    const int j = e / LD, i = e % LD;
    P[e] = i < TS ? (i == j ? 20.0 : 1.0 / (1 + i + j)) : 0.0;
  }
  if (threadIdx.x == 0) done = 0;
  __syncthreads();
  if (w == 0) {
    int cnt = 0;
    for (int it = 0; it < iters; ++it) cnt += wave_chol_tile<double, LD>(P, Lt, Li, 1e-300, nullptr);
    __hip_atomic_store(&done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cnt != 0 || Lt[lane] == -1.0) out[blockIdx.x] = Lt[lane] + Li[lane];
  } else {
    const double a = 1.0 + lane * 1e-3, b = 1.0 - (lane & 7) * 1e-3;
    d4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < MAX_TRIPS; ++t) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = mfma(a, b, acc[i]);
      if (__hip_atomic_load(&done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    if (s == -1.0) out[blockIdx.x] = s;
  }
}

}  // namespace

void launch_ceiling_chol(hipStream_t st, bool beside, int grid, int iters, double* out) {
  hipLaunchKernelGGL(k_chol_latency, dim3(grid), dim3(beside ? 320 : 64), 0, st, iters, out);
}

void launch_ceiling_mfma(hipStream_t st, bool fp32, int grid, int iters, double* out) {
  if (fp32) hipLaunchKernelGGL(k_mfma_peak<float>, dim3(grid), dim3(256), 0, st, iters, out);
  else hipLaunchKernelGGL(k_mfma_peak<double>, dim3(grid), dim3(256), 0, st, iters, out);
}

void launch_ceiling_read(hipStream_t st, const double* buf, long long n, int grid, double* out) {
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, st,
                     reinterpret_cast<const dv2*>(buf), n / 2, out);
}

}  // namespace ahlp
