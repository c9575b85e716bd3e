// Host-callable launchers of the device kernels (one stream each).
#pragma once

#include "common.h"

namespace ahlp {

// factorization (k_factor.hip)
// D = (z/x + q + rho)^-1 (q: the bounds' W/S, or null)
void launch_prep(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                 long long d0off, const double* x, const double* z, const double* q, double rho,
                 double* Dp, double* xs, double* zs, DevInfo* info);
template <typename T>
void launch_syrk(hipStream_t st, const BlockInfo* blk, const int4* items, int nitems,
                 const T* A, const double* Dp, T* LB, double delta);
template <typename T>
// nb: width of the border section (global rows, then x_0)
void launch_link(hipStream_t st, const BlockInfo* blk, const int2* items, int nitems, int nb,
                 const double* A, const double* C, const int* lptr, const int* lcol,
                 const double* lval, const double* Dp, T* LB, double* PQ);
// Block factorization of the blocks order[0..n) (bordered Cholesky giving L_i
// and W_i', then the FP64 Schur contributions PQ): the panel kernel for
// blocks whose bordered tile rows fit (block_factor_panel_fits), the
// column-at-a-time kernel plus a product pass for any height.  max_rt: the
// largest bordered tile-row count among the n blocks; max_kt (if >= 0) an
// upper bound on their link-column tile counts, which sizes the LDS for the
// Schur contribution.
template <typename T>
void launch_block_factor_panel(hipStream_t st, const BlockInfo* blk, const int* order, int n,
                               int max_rt, T* LB, T* LINV, double* PQ, DevInfo* info,
                               int waves = 4, int max_kt = -1);
template <typename T>
void launch_block_factor_col(hipStream_t st, const BlockInfo* blk, const int* order, int n,
                             int max_rt, T* LB, T* LINV, double* PQ, DevInfo* info);
bool block_factor_panel_fits(int rt);    // the four-wave form
bool block_factor_panel8_fits(int rt);   // the eight-wave form
// a1-a5 for the panel bucket in one persistent launch (link columns, SYRK,
// panel factorization and Schur contributions); num_cu: compute units.
template <typename T>
void launch_factor_fused(hipStream_t st, const BlockInfo* blk, const int* order, int n,
                         int max_rt, int* queue, int nb, const T* Aw, const double* A,
                         const double* C, const int* lptr, const int* lcol, const double* lval,
                         const double* Dp, T* LB, T* LINV, double* PQ, double delta,
                         DevInfo* info, int num_cu);
bool factor_fused_fits(int rt, int mt);
// T, E (l_j x nb) and S00 (nb x nb) of S; F0: the extended (nl + ng) x n0
// x_0 coupling (link rows, then the global rows' Wg0), or null; F0L: the same
// pointer, or null when its link rows are zero
void launch_assemble(hipStream_t st, const BlockInfo* blk, int N, int nb, int n0, long long nl,
                     const int* lsz, const long long* tdoff, const long long* tooff,
                     const long long* eoff, const double* PQ, const double* F0L,
                     const double* F0, const long long* loff, double delta, const double* D0,
                     double* Td, double* To, double* E, double* S00, double* thrT);
void launch_convert_f32(hipStream_t st, long long n, const double* src, float* dst);

// Schur complement (k_chain.hip).  Its border (called n0 in the Schur
// kernels) is the global rows' duals (the first ng entries, a positive
// definite part) followed by x_0 (negative definite).
struct ChainArgs {
  int P, G, n0, ng;
  const int* l;            // [P]
  const long long* tdoff;  // [P]    l_j^2 blocks (T_jj, L_j, L_j^-1)
  const long long* tooff;  // [P-1]  l_{j+1} x l_j blocks (T_{j+1,j}, Yn_j)
  const long long* eoff;   // [P]    l_j x n0 blocks (E_j, G_j)
  const long long* zoff;   // [P]    l_{left separator} x l_j blocks (Z_j)
  const long long* suboff; // [G]    separator couplings
  const int2* seg;         // [G]    interior pairs [a, b)
  const double* Td; const double* To; const double* E; const double* S00; const double* thrT;
  double* CL; double* CLi; double* CYn; double* CZ; double* CG; double* CSub;
  double* Lb; double* Lbi; double* S00w;
  double* segout;          // per segment: SEG_STRIDE doubles
  int lmax;
  DevInfo* info;
};

constexpr int SEG_STRIDE = 3 * LMAX * LMAX + 2 * LMAX * N0MAX + N0MAX * N0MAX;
// segment output slot layout (compact, leading dimension = actual size)
__device__ inline double* so_diagL(double* s) { return s; }
__device__ inline double* so_EL(double* s) { return s + LMAX * LMAX; }
__device__ inline double* so_diagR(double* s) { return s + LMAX * LMAX + LMAX * N0MAX; }
__device__ inline double* so_ER(double* s) { return s + 2 * LMAX * LMAX + LMAX * N0MAX; }
__device__ inline double* so_off(double* s) { return s + 2 * LMAX * LMAX + 2 * LMAX * N0MAX; }
__device__ inline double* so_S00(double* s) { return s + 3 * LMAX * LMAX + 2 * LMAX * N0MAX; }

// rhs s and solution u: [pairs (offsets loff) | x_0 (offset nl)]; w: forward
// intermediate in the same layout.
struct ChainSolveArgs {
  ChainArgs c;
  const long long* loff;
  long long nl;
  const double* s;
  double* w;
  double* u;
  double* segrhs;      // per segment: 2*LMAX + N0MAX doubles (dsL, dsR, ds0)
};
constexpr int SEGRHS_STRIDE = 2 * LMAX + N0MAX;


// Tile path (pairs of at most 16 rows, at most 64 linking variables).
// Block cyclic reduction of T and the border (k_bcr.hip), pairs of <= 16 rows,
// n0 <= 64.  Tiles are 16x16 column-major, padded.
struct BcrArgs {
  int P, n0, t0, ng;                              // n0: border width, ng of it global rows
  int tp;                                         // tiles per pair side (1 or 2)
  const int* l;
  const long long* tdoff;
  const long long* tooff;
  const long long* eoff;
  const double* Td; const double* To; const double* E; const double* S00; const double* thrT;
  double* BD; double* BC; double* BEt;            // working tiles (P tp^2, P tp^2, P tp t0)
  double* FLi; double* FXL; double* FXR; double* FGt;   // factor tiles (same counts)
  double* FLb; double* FLbi;                      // border factor, t0*t0 tiles each
  double* s00part;                                // per chunk of pairs: t0*t0 tiles
  DevInfo* info;
};
struct BcrSolveArgs {
  BcrArgs c;
  const long long* loff;
  long long nl;
  const double* s;       // right-hand side (exact pair layout, then n0 border values)
  double* u;             // solution, same layout
  double* r; double* w; double* up;   // padded pair vectors, 16 tp per pair
  double* pb;            // border partials Z_j' w_j, 16*t0 per pair
  double* u0p;           // border solution, 16*t0
};
// tiles per pair side of the cyclic-reduction path for these sizes (1 or 2),
// 0 if it does not apply
int bcr_tiles(int lmax, int n0);
void launch_bcr_factor(hipStream_t st, const BcrArgs& c, int nparts, int chunk);
void launch_bcr_solve(hipStream_t st, const BcrSolveArgs& a);
void set_bcr_smem_limits();
// device ceilings (k_ceiling.hip): grid workgroups of 256 threads
void launch_ceiling_mfma(hipStream_t st, bool fp32, int grid, int iters, double* out);
void launch_ceiling_read(hipStream_t st, const double* buf, long long n, int grid, double* out);
// grid workgroups of one factoring wave (and four MFMA-streaming waves if beside)
void launch_ceiling_chol(hipStream_t st, bool beside, int grid, int iters, double* out);
// two-tile pairs (k_bcr2.hip): the reduction of T down to the final pair, and
// the whole solve
void launch_bcr2_reduce(hipStream_t st, const BcrArgs& c);
void launch_bcr2_solve(hipStream_t st, const BcrSolveArgs& a);
void set_bcr2_smem_limits();

size_t chain_factor_smem(int lmax, int n0);
void launch_chain_factor(hipStream_t st, const ChainArgs& c);
void launch_chain_solve(hipStream_t st, const ChainSolveArgs& a);
void set_chain_smem_limits(size_t bytes);

// solve phase and glue (k_solve.hip)
void launch_pad_x(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                  long long d0off, const double* x, double* xp, const double* scale);
void launch_pad_y(hipStream_t st, const BlockInfo* blk, int N, const double* y, double* yp);
void launch_rhx(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                long long d0off, const double* rx, const double* rz, const double* xs,
                const double* Dp, double* rhx, double* vx);
// Row pass for up to RV_MAX vectors (one read of A):
//   out_k = base_k + alpha_k (A_i v_k [+ C_i v_k,0]);  chain_k: base_k = output k-1 (same row)
constexpr int RV_MAX = 3;
struct RowsArgs {
  int nv;
  const double* v[RV_MAX];      // padded x-space vectors (x_0 part at d0off)
  const double* base[RV_MAX];   // canonical y-space base, or null
  double alpha[RV_MAX];
  double* out[RV_MAX];
  int with_C[RV_MAX];           // include the C_i x_0 columns
  int padded[RV_MAX];           // output in padded v-space (rows >= m_i set to 0) or canonical
  int chain[RV_MAX];
};
// w = D (a b) / x (padded x-space; a, b canonical, null a: w = D / x); x_0 part zero
void launch_wscaled(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                    long long d0off, const double* a, const double* b, const double* xs,
                    const double* Dp, double* w);
// out = t - smu * a + b over n values
// out = t - smu a + b; smu from *smu_dev when that is not null
void launch_combine(hipStream_t st, long long n, const double* t, double smu, const double* a,
                    const double* b, double* out, const double* smu_dev = nullptr);
// scal[s_out] = (mu_aff / mu)^3 mu with mu = scal[s_xz] / n, mu_aff = scal[s_muaff] / n;
// with bounds (s_sw >= 0) both also take the (s, w) products, scal[s_sw] and
// scal[s_muaff_sw], and n counts the bounded variables too
void launch_sigma_mu(hipStream_t st, double* scal, long long n, int s_xz, int s_muaff, int s_out,
                     int s_sw = -1, int s_muaff_sw = -1);
// r = max(clip(v, lo, hi) - v, -hi), v = (x + at_p dx)(z + at_d dz), [lo, hi] =
// [beta_min, beta_max] * smu[0] (a Gondzio corrector's right-hand side)
void launch_gondzio_rhs(hipStream_t st, long long n, const double* x, const double* z,
                        const double* dx, const double* dz, double at_p, double at_d,
                        const double* smu, double beta_min, double beta_max, double* r);
// up to four step updates in one launch: x[v] += min(1, eta ratio[v][0]) d[v]
struct StepSet {
  int cnt;
  long long n[6];
  const double* ratio[6];
  const double* d[6];
  double* x[6];
};

// Upper bounds inside the interior-point iteration.  A bounded variable
// (finite ub) has the slack s = u - x and its dual w; eliminating ds and dw
// leaves the Newton system with Q = W/S in its (x, x) block, whose x right-hand
// side is r_d + S^-1 (r_sw - W r_u).  ub == nullptr: no bounds (every other
// field unused).  s, w, q, ru are zero off the bounded variables.
struct BndArgs {
  const double* ub;      // [n_tot] upper bounds, +inf where none
  const double* s;       // slacks
  const double* w;       // their duals
  const double* q;       // w / s
  const double* ru;      // u - x - s
  const double* rdt;     // the predictor's x right-hand side r_d - w - q r_u
  const double* dsa;     // the predictor's ds, dw (the corrector's products)
  const double* dwa;
  const double* smu;     // device scalar sigma mu (corrector)
  double* ds;            // recovered ds, dw of the direction being checked
  double* dw;
  int mode;              // 0: predictor (r_sw = -SWe), 1: corrector
};
void launch_steps(hipStream_t st, double eta, const StepSet& s);
void launch_rows_multi(hipStream_t st, const BlockInfo* blk, const int2* rowtiles, int nrt,
                       const double* A, const double* C, long long d0off, const RowsArgs& ra);
void launch_rows(hipStream_t st, const BlockInfo* blk, const int2* rowtiles, int nrt,
                 const double* A, const double* C, const double* xp, long long d0off,
                 const double* base, double alpha, int with_C, int padded_out, double* out);
// the dual rows after the blocks (link rows, then global rows):
// out = base + alpha (F xp [+ F0 x0]); F0 the extended (nl + ng) x n0 coupling,
// F0L the same or null when its link rows are zero
void launch_linkrows(hipStream_t st, const BlockInfo* blk, int P, int ng, int n0,
                     const int* lsz, const long long* loff, long long nl, const int* lptr,
                     const int* lcol, const double* lval, const int* gptr, const int* gidx,
                     const double* gval, const double* xp, const double* x0, const double* F0,
                     const double* F0L, const double* base, double alpha, double* out);
// Optional fused output of the column pass (mode 2): dz = (rz - zs dx) / xs
struct DzArgs {
  const double* rz; const double* zs; const double* xs; double* dz;
};
void launch_cols(hipStream_t st, const BlockInfo* blk, const int2* coltiles, int nct,
                 const double* A, const double* yp, const double* yL, const int* cptr,
                 const int* crow, const double* cval, int mode, const double* cvec,
                 const double* zvec, const double* Dp, double* gout, double* out,
                 const DzArgs& dzv = DzArgs{});
void launch_ccols(hipStream_t st, const BlockInfo* blk, const int2* ctiles, int nctile, int n0,
                  const double* C, const double* yp, double* part);
// F0 rows below f0first are zero (skipped)
void launch_x0_sum(hipStream_t st, int N, int n0, long long nl, long long f0first,
                   const double* part, const double* F0, const double* yL, int mode,
                   const double* cvec, const double* zvec, long long x0off, double* gout,
                   double* out);
template <typename T>
void launch_block_fwd(hipStream_t st, const BlockInfo* blk, int N, int max_rt, const T* LB,
                      const T* LINV, const double* tin, double* tv, double* qn);
template <typename T>
void launch_block_bwd(hipStream_t st, const BlockInfo* blk, int N, int nb, long long nl,
                      int max_rt, const T* LB, const T* LINV, const double* v, const double* u,
                      double* dy, double* dyp);
void launch_schur_rhs(hipStream_t st, const BlockInfo* blk, int N, int nb, const int* lsz,
                      const long long* loff, long long nl, const double* qn, const double* rhx0,
                      double* s);
void launch_solve_tail(hipStream_t st, int N, int n0, long long nl, long long f0first,
                       const double* part, const double* F0, const double* u, long long x0off,
                       long long mblk, double* gout, double* dx, const DzArgs& dzv, double* dy);
// ex = rx - g - dz (+ q dx where b.q is given: the (x, x) block -Q of a
// factorization with bounds); with bounds (b.ub) it also recovers b.ds, b.dw
// from dx and forms w2 = D (dx dz / x - ds dw / s)
void launch_check_prep(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                       long long d0off, const double* rx, const double* rz, const double* g,
                       const double* dx, const double* dz, const double* xs, const double* zs,
                       const double* Dp, double* ex, double* ez, double* xp, double* w2p,
                       const BndArgs& b);
// with bounds (b.ub): the predictor's x right-hand side rdt = r_d - w - q r_u
// (written to rdt_out) replaces r_d, and w1 = D (1/x - 1/s)
void launch_resid_prep(hipStream_t st, const BlockInfo* blk, int N, int n0, long long x0off,
                       long long d0off, const double* x, const double* z, const double* rd,
                       const double* xs, const double* Dp, double* rzv, double* rhx, double* vx,
                       double* w1p, double* xp, const BndArgs& b, double* rdt_out);
void launch_axpy(hipStream_t st, long long n, double a, const double* x, double* y);
// mode 0: out = zs * v; mode 1: out = v / zs (the diagonal scalings that turn
// the transposed Newton solve into a Newton solve)
void launch_adj_scale(hipStream_t st, long long n, int mode, const double* zs, const double* v,
                      double* out);
void launch_dz(hipStream_t st, long long n, const double* rz, const double* zs, const double* xs,
               const double* dx, double* dz);
void launch_rd(hipStream_t st, long long n, const double* c, const double* g, const double* z,
               double* rd);
void launch_res_x(hipStream_t st, long long n, const double* rx, const double* rz,
                  const double* g, const double* dx, const double* dz, const double* xs,
                  const double* zs, double* ex, double* ez);
void launch_copy(hipStream_t st, long long n, const double* src, double* dst);
// rz = -x z (mode 0) or smu - x z - dxa dza (mode 1); smu from *smu_dev when not null.
// With bounds (b.ub, mode 1) also the corrector's x right-hand side
// rxc = rdt + (smu - dsa dwa) / s on the bounded variables
void launch_rz(hipStream_t st, long long n, int mode, const double* x, const double* z,
               const double* dxa, const double* dza, double smu, double* rz,
               const double* smu_dev = nullptr, const BndArgs* b = nullptr, double* rxc = nullptr);
// bounds at an iterate: ru = u - x - s, q = w / s, zw = z - w (0, 0, z off the
// bounded variables); flags s <= 0, w <= 0 or non-finite ones in info
void launch_bnd_prep(hipStream_t st, long long n, const double* ub, const double* x,
                     const double* z, const double* s, const double* w, double* ru, double* q,
                     double* zw, DevInfo* info);
// start: on the bounded variables s = u - x, w = max(-z, 0), z = max(z, 0),
// elsewhere s = w = 0; sm, wm = s, w there and +inf elsewhere (for minima)
void launch_bnd_start(hipStream_t st, long long n, const double* ub, const double* x, double* z,
                      double* s, double* w, double* sm, double* wm);
// x += a, z += c everywhere; s += a, w += c on the bounded variables; then sm,
// wm as in launch_bnd_start
void launch_bnd_shift(hipStream_t st, long long n, const double* ub, double a, double c,
                      double* x, double* z, double* s, double* w, double* sm, double* wm);
void launch_fill(hipStream_t st, long long n, double v, double* dst);
void launch_addscalar(hipStream_t st, long long n, double v, double* dst);
void launch_reduce(hipStream_t st, int op, long long n, const double* a, const double* b,
                   const double* c, const double* d, double s1, double s2, double* partial,
                   double* out);

struct RedSpec {
  int op, slot;          // operation, output slot
  long long n;
  const double* a; const double* b; const double* c; const double* d;
  double s1, s2;
  const double* ps1;     // if set (op RED_MUAFF): s1 = min(1, *ps1), s2 = min(1, *ps2),
  const double* ps2;     // read from the device (results of an earlier reduction)
};
constexpr int MAXRED = 16;
struct MultiRed {
  int nred;
  RedSpec r[MAXRED];
  double* partial;       // [MAXRED * RED_PARTIALS]
  double* out;
};
void launch_mreduce(hipStream_t st, const MultiRed& m);

// RED_RATIO2: the ratio test over two pairs, min over i of -a/b (b < 0) and -c/d (d < 0)
enum RedOp { RED_DOT = 0, RED_MAXABS = 1, RED_RATIO = 2, RED_MUAFF = 3, RED_MAXSUM = 4, RED_MIN = 5,
             RED_RATIO2 = 6 };
constexpr int RED_PARTIALS = 256;

// ---- static workspace (noalloc.hip)
// Size of the per-device static array that ahlp_kkt_solve_noalloc works in.
constexpr size_t SCRATCH_BYTES = size_t(32) << 20;
// Resolves the array's device address on `device` (which must be current) and
// keeps it; later calls return at once.  hipSuccess or the HIP error.
hipError_t scratch_setup(int device);
// The kept address for `device`, or nullptr before a successful setup.
double* scratch_device_ptr(int device);

}  // namespace ahlp
