// Shared definitions of libahlp's device code and host orchestration.
//
// Device data layout (all dense block matrices): 16x16 tiles, column-major
// inside a tile (element (i, k) at k*16 + i), 256 elements per tile.  With this
// layout the operands of a 16x16x4 MFMA are contiguous: for k-step s a lane l
// reads element 64*s + l of the tile, for both the A operand (rows of C) and the
// B operand of a product with a transposed tile (C += X Y').  Block rows are
// padded to a multiple of 16 with zero rows, block columns likewise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ahlp {

constexpr int TS = 16;          // tile edge
constexpr int TE = 256;         // elements per tile
constexpr double PIVOT_REL = 1e-30;
constexpr double PIVOT_BIG = 1e128;
constexpr int LMAX = 64;        // largest link pair handled by the chain kernels
constexpr int N0MAX = 128;      // largest border of S: global rows plus linking variables

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));

// 16-byte load of data that a pass reads once (the blocks of A in the row and
// column passes): nontemporal, so the caches do not keep it for reuse that
// never comes (measured on gfx950: 5.8-6.0 TB/s against 5.3 for plain loads
// when streaming 512 MiB).
__device__ __forceinline__ dv2 ld_stream2(const dv2* p) { return __builtin_nontemporal_load(p); }

// Per-block geometry, offsets and section layout (host computes, device reads).
struct BlockInfo {
  int m, n;          // real rows / columns of A_i
  int mt, nt;        // tile counts of the padded block (16 mt x 16 nt)
  int kt, rt;        // link-column tiles (kp = 16 kt) and bordered tile rows mt + kt
  int lL, lR;        // real rows of the left pair (i-1) and right pair (i); 0 at the ends
  int ktL, ktR, kt0; // tiles of the left, right and border sections of the link columns;
                     // the border holds the ng global rows, then the n0 x_0 columns
  int ng, kc0;       // global rows at the start of the border; tiles of C_i (n0 columns)
  int pairL, pairR;  // pair indices, -1 when absent
  int csr_off;       // this block's kp+1 link-row pointers start here in linkptr
  int csc_off;       // this block's n+1 link-column pointers start here in lcolptr
  long long xoff, yoff;   // offsets in the canonical x and y vectors
  long long dpoff;        // offset in the padded D vector (multiple of 16)
  long long aoff;         // A tiles (mt x nt, row-of-tiles major)
  long long coff;         // C tiles (mt x kc0)
  long long lboff;        // bordered factor: lower-trapezoid tile columns, packed
  long long linvoff;      // mt inverted diagonal tiles of L_i
  long long pqoff;        // kt x kt tiles of the Schur contribution F D F' - W'W
  long long loffL, loffR; // start of the left / right pair inside y_L (-1 if none)
  long long voff;         // offset of the block in padded block-row vectors (sum 16 mt)
  long long qoff;         // offset in link-column vectors (sum 16 kt)
};

// Column c of the bordered factor holds tile rows c..rt-1 contiguously.
__host__ __device__ inline long long lb_tile(const BlockInfo& b, int r, int c) {
  long long colstart = (long long)c * b.rt - (long long)c * (c - 1) / 2;
  return b.lboff + (colstart + (r - c)) * TE;
}
__host__ __device__ inline long long lb_tiles(int mt, int rt) {
  return (long long)mt * rt - (long long)mt * (mt - 1) / 2;
}
__host__ __device__ inline long long a_tile(const BlockInfo& b, int I, int K) {
  return b.aoff + ((long long)I * b.nt + K) * TE;
}
__host__ __device__ inline long long c_tile(const BlockInfo& b, int I, int Q) {
  return b.coff + ((long long)I * b.kc0 + Q) * TE;
}
__host__ __device__ inline long long pq_tile(const BlockInfo& b, int r, int c) {
  return b.pqoff + ((long long)r * b.kt + c) * TE;
}

// Link-column section of row q (0 <= q < 16 kt): 0 left pair, 1 right pair,
// 2 border (global rows, then x_0); *idx receives the index inside the
// section and *real whether it is a real (not padding) row.  nb: the border's
// width, ng + n0.
__host__ __device__ inline int link_section(const BlockInfo& b, int q, int* idx, int nb, bool* real) {
  int qL = TS * b.ktL, qR = TS * b.ktR;
  if (q < qL) { *idx = q; *real = q < b.lL; return 0; }
  q -= qL;
  if (q < qR) { *idx = q; *real = q < b.lR; return 1; }
  q -= qR;
  *idx = q; *real = q < nb; return 2;
}
// Whether link-column row q of a section is a sparse row of F_i (a link row
// or a global row) rather than a column of C_i.
__host__ __device__ inline bool link_is_row(const BlockInfo& b, int sec, int idx) {
  return sec < 2 || idx < b.ng;
}

// D += A B for a 16x16x4 block: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the result follows acc_index below.
__device__ inline d4 mfma(double a, double b, d4 c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
#else
  return c;
#endif
}
__device__ inline f4 mfma(float a, float b, f4 c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
#else
  return c;
#endif
}

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 type; };
template <> struct Acc<float> { typedef f4 type; };

// Row of accumulator element r of lane l (the column is always l%16).  The two
// 16x16x4 MFMA variants differ: FP32 returns rows 4*(l/16) + r, FP64 returns
// rows 4*r + l/16 (checked on gfx950 with a one-wave layout probe).
template <typename T> __host__ __device__ inline int acc_row(int lane, int r);
template <> __host__ __device__ inline int acc_row<double>(int lane, int r) { return 4 * r + (lane >> 4); }
template <> __host__ __device__ inline int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
// Index inside a column-major tile of accumulator element r of lane l.
template <typename T> __host__ __device__ inline int acc_index(int lane, int r) {
  return (lane & 15) * TS + acc_row<T>(lane, r);
}

// Status/info word shared by all kernels of one handle.
struct DevInfo {
  int pivots;       // pivots replaced by the pivot rule
  int nonfinite;    // x or z not finite / not positive at factor
};

// Cross-lane sums on the VALU (DPP moves within a 16-lane row, permlane
// swaps across rows) instead of LDS-pipe permutes.  Each gives every lane the
// additions of the xor butterfly x += shfl_xor(x, s) over its strides, in the
// same order, so the results are bitwise the same.  The controls used here
// (quad permutations, row mirrors) give every lane a source, so a move needs
// no old value.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  union { double d; int i[2]; } u, o;
  u.d = v;
  o.i[0] = __builtin_amdgcn_mov_dpp(u.i[0], CTRL, 0xF, 0xF, false);
  o.i[1] = __builtin_amdgcn_mov_dpp(u.i[1], CTRL, 0xF, 0xF, false);
  return o.d;
}
// strides 1, 2, 4, 8: the sum over the lane's 16-lane row.  After the two
// quad steps every lane of a quad holds the same value, so the half-row and
// row mirrors read the same values as the xor-4 and xor-8 partners.
__device__ __forceinline__ double row_sum16(double x) {
  x += dpp_mov<0xB1>(x);    // quad_perm [1,0,3,2]: lane ^ 1
  x += dpp_mov<0x4E>(x);    // quad_perm [2,3,0,1]: lane ^ 2
  x += dpp_mov<0x141>(x);   // row_half_mirror: the other quad of the half row
  x += dpp_mov<0x140>(x);   // row_mirror: the other half row
  return x;
}
// x_l + x_(l ^ S) for S = 16 or 32: the swap leaves the two values of each
// lane pair in its two outputs, whose sum is the same in both lanes
template <int S>
__device__ __forceinline__ double pair_sum(double x) {
  union { double d; unsigned i[2]; } u, a, b;
  u.d = x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if constexpr (S == 16) {
      const auto r = __builtin_amdgcn_permlane16_swap(u.i[h], u.i[h], false, false);
      a.i[h] = r[0];
      b.i[h] = r[1];
    } else {
      const auto r = __builtin_amdgcn_permlane32_swap(u.i[h], u.i[h], false, false);
      a.i[h] = r[0];
      b.i[h] = r[1];
    }
  }
  return a.d + b.d;
}
// strides 16, 32: the sum over lanes l, l ^ 16, l ^ 32, l ^ 48
__device__ __forceinline__ double col_sum4(double x) { return pair_sum<32>(pair_sum<16>(x)); }

}  // namespace ahlp
