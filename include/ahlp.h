/*
 * ahlp.h -- C ABI of libahlp: the per-iteration Newton-system solve of a
 * primal-dual interior-point method for arrowhead linear programs with local
 * linking structure, on one AMD MI355X (gfx950).
 *
 * The LP (Sec. 2.2 standard form with the block structure of Sec. 3.2,
 * equality rows, local two-link constraints and global linking rows of
 * Sec. 3.3):
 *
 *     min c'x   s.t.  A_i x_i + C_i x_0                        = b_i    i = 0..N-1
 *                     FR_j x_j + FL_j x_{j+1} + F0_j x_0       = b_Lj   j = 0..N-2
 *                     Wg_0 x_0-block + .. + Wg_{N-1} x_{N-1}-block + Wg0 x_0 = b_G
 *                     x >= 0
 *
 * (A_i is the paper's B_i, C_i its A_i, FR_j its local block F_j, FL_j its F'_j,
 * F0 the local part of its F_0; Wg_i and Wg0 are rows of its F and F_0 with
 * global support, which the Schur complement keeps in its dense border, the
 * dense layer of Sec. 4.1.)  Canonical vector order:
 *     x, z = [x_0-block .. x_{N-1}-block, x_0]       length n_tot = sum n_i + n0
 *     y    = [y_0 .. y_{N-1}, y_L(pair 0) .. y_L(pair N-2), y_G]
 *                                                   m_tot = sum m_i + sum l_j + ng
 *
 * Conventions for every call:
 *   - Status codes: 0 on success, negative on error, positive for warnings whose
 *     outputs are valid.  On error ahlp_last_error() returns a message
 *     (thread-local; valid until the next call on the same thread).
 *   - "device" pointers are HIP device memory on the device that was current
 *     when the problem was created; "host" pointers are ordinary CPU memory.
 *   - Calls are stream ordered on the given stream (0 = the null stream).
 *     ahlp_kkt_factor and ahlp_kkt_solve return after enqueueing unless noted;
 *     ahlp_problem_create and ahlp_ipm_solve synchronize the stream.
 *   - A handle is not thread safe; distinct handles are independent.
 *   - Results are bitwise reproducible for the same inputs, device and stream
 *     (fixed-order reductions; no floating-point atomics).
 */
#ifndef AHLP_H
#define AHLP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ahlp_problem_s* ahlp_problem_t;   /* opaque, library owned */

typedef enum {
  AHLP_OK = 0,
  AHLP_EINVAL = -1,    /* null or inconsistent arguments, unsupported sizes     */
  AHLP_ENOMEM = -2,    /* device or host allocation failed                        */
  AHLP_EHIP = -3,      /* HIP runtime or launch error                             */
  AHLP_ESTATE = -4,    /* call out of order (e.g. solve before factor)            */
  AHLP_ENUMERIC = -5,  /* non-finite data, or x <= 0 / z <= 0 handed to factor     */
  AHLP_WMAXITER = 1,   /* interior-point loop stopped at max_iter                  */
  AHLP_WSTALL = 2      /* interior-point step length collapsed                     */
} ahlp_status_t;

typedef enum {
  AHLP_FP64 = 0,         /* every stage in FP64                                    */
  AHLP_FP32_REFINE = 1   /* block SYRK / Cholesky / TRSM in FP32 MFMA with FP32
                            accumulation; Schur assembly and factorization,
                            residuals and refinement in FP64                        */
} ahlp_precision_t;

/* Problem data for ahlp_problem_create.  All arrays are HOST memory, FP64,
 * row-major per block, blocks concatenated in order.  Limits: N >= 1,
 * 1 <= m_i <= n_i, 0 <= l_j <= min(n_j, n_{j+1}, 64), 0 <= n0, 0 <= ng,
 * ng + n0 <= 128 (the border of the Schur complement), and
 * every bordered block fits the LDS of one workgroup: with rt_i the 16-row
 * tiles of m_i plus those of l_{i-1}, l_i and ng + n0 (each rounded up),
 * (rt_i + 1) * 16 * 17 * 8 bytes <= the device's LDS per workgroup (160 KiB
 * on gfx950: rt_i <= 74, blocks of up to about 1,180 rows with their links).
 * The problem is handed over in host memory because create repacks it into
 * the library's tile layout on the host, once (a reading of the boundary:
 * every per-iteration call takes device pointers). */
typedef struct {
  int32_t N;              /* number of diagonal blocks                              */
  int32_t n0;             /* number of linking variables x_0                        */
  const int32_t* m;       /* [N]   rows of A_i                                      */
  const int32_t* n;       /* [N]   columns of A_i                                   */
  const int32_t* l;       /* [N-1] local linking rows between blocks j and j+1 (may
                             be NULL when N == 1)                                   */
  const double* A;        /* concat_i A_i   (m_i x n_i)                             */
  const double* C;        /* concat_i C_i   (m_i x n0); NULL iff n0 == 0             */
  const double* FR;       /* concat_j FR_j  (l_j x n_j)      block j's part of pair j */
  const double* FL;       /* concat_j FL_j  (l_j x n_{j+1})  block j+1's part        */
  const double* F0;       /* (sum l) x n0 coupling of link rows to x_0; NULL = 0     */
  const double* b;        /* [m_tot]: block rows, link rows, global rows             */
  const double* c;        /* [n_tot]                                                 */
  int32_t ng;             /* global linking rows (0: none; then Wg, Wg0 unused)      */
  const double* Wg;       /* concat_i Wg_i  (ng x n_i)   block i's part of them      */
  const double* Wg0;      /* ng x n0 their x_0 part; NULL = 0                         */
  const double* ub;       /* [n_tot] upper bounds x <= u (Sec. 3.2), +inf where none, */
                          /* finite ones > 0; NULL = none.  ahlp_ipm_solve keeps them */
                          /* inside the iteration (a slack s = u - x and a dual w per  */
                          /* bounded variable, see ahlp_kkt_factor_bounded)           */
} ahlp_problem_desc_t;

/* Regularization of the factorization (a reading: the paper leaves pivot
 * handling to its sparse solvers).  With D = (Z/X + rho)^-1 the block matrices
 * are M_i = A_i D_i A_i' + delta I and the link part of the Schur complement
 * gets + delta I. */
typedef struct {
  ahlp_precision_t precision;
  double rho;             /* primal regularization, >= 0                           */
  double delta;           /* dual regularization, >= 0                             */
} ahlp_factor_opts_t;

typedef struct {
  double tol;             /* stop when relgap, pinf and dinf are all <= tol (1e-8)   */
  int32_t max_iter;       /* 100                                                     */
  double eta;             /* step damping 0.99                                       */
  double rho, delta;      /* 1e-8, 1e-6                                              */
  int32_t max_refine;     /* refinement corrections per solve (5)                    */
  double refine_tol;      /* backward-error target (1e-10)                           */
  ahlp_precision_t precision;
  double mu_switch;       /* FP32 mode: switch to FP64 blocks for good once mu < this */
  int32_t start;          /* 0 = Mehrotra starting point, 1 = use x, y, z as given    */
  int32_t verbose;        /* 1 = one log line per iteration on stderr                */
  int32_t timing;         /* 1 = record per-stage device times (HIP events); 2 = the  */
                          /* factorization stages PREP, SYRK, FACTOR, SCHUR only      */
                          /* (fewer events, so less perturbation of the run)          */
  double fp32_accept;     /* FP32 mode: a direction from FP32 factors is accepted      */
                          /* once |r - K d|_inf <= fp32_accept * mu (inexact Newton;   */
                          /* 0.1; 0 = only the refine_tol backward error).  FP32 that   */
                          /* cannot reach either test switches the run to FP64 and     */
                          /* the iteration is redone with FP64 factors.  < 0: the      */
                          /* plain rule of FP64 factors (refine until refine_tol or    */
                          /* max_refine corrections, then keep the last direction)     */
  int32_t graph;          /* 1 = capture the three parts of an iteration between its */
                          /* host reads (factorization + predictor, corrector, step  */
                          /* + residuals) as hipGraphs once and replay them (results */
                          /* identical to 0); ignored when timing != 0.  The solve   */
                          /* then runs on a library stream ordered after and before  */
                          /* the caller's stream.  0 by default                      */
  int32_t gondzio;        /* at most this many Gondzio centrality correctors per     */
                          /* iteration after Mehrotra's corrector (0 by default)      */
} ahlp_ipm_opts_t;

/* Stage indices of ahlp_ipm_result_t.t_stage_ms / n_stage. */
enum {
  AHLP_ST_PREP = 0,       /* D-scaling, link columns (a1)                            */
  AHLP_ST_SYRK = 1,       /* M_i = A_i D_i A_i' (a2)                                 */
  AHLP_ST_FACTOR = 2,     /* Cholesky of M_i and W_i = L_i^-1 B_i (a3, a4)            */
  AHLP_ST_SCHUR = 3,      /* W_i' W_i and assembly of S (a5)                          */
  AHLP_ST_TFACTOR = 4,    /* block-tridiagonal + border factorization of S (a6)       */
  AHLP_ST_SOLVE = 5,      /* solve phase (a7)                                         */
  AHLP_ST_RESID = 6,      /* residuals, reductions, refinement residuals (a8)         */
  AHLP_ST_AROWS = 7,      /* each row pass out = base + A v over the dense blocks,    */
                          /* timed alone; it also counts inside SOLVE and RESID       */
  AHLP_ST_COUNT = 8
};

typedef struct {
  int32_t status;         /* ahlp_status_t of the run                                */
  int32_t iterations;     /* factorizations after the starting point                 */
  int32_t refine_steps;   /* refinement corrections, all solves                      */
  int32_t pivots_modified;/* pivots replaced by the pivot rule                        */
  int32_t fp32_iterations;/* iterations whose blocks were factored in FP32           */
  double primal_obj, dual_obj, rel_gap, rel_pinf, rel_dinf, mu;
  double max_bkerr;       /* largest backward error after refinement                 */
  double t_total_ms;      /* wall time of the call                                   */
  double t_stage_ms[AHLP_ST_COUNT];   /* summed device time per stage (timing=1)     */
  int32_t n_stage[AHLP_ST_COUNT];     /* number of timed launches per stage         */
  double rows_bytes;      /* algorithmic HBM bytes of the timed row passes          */
                          /* (AHLP_ST_AROWS): A and C read, vectors read and written */
  int32_t correctors;     /* Gondzio correctors kept over the whole run             */
  double start_bkerr[2];  /* backward errors of the two starting-point solves       */
                          /* after refinement (-1 with opts->start == 1)            */
  double t_stage32_ms[AHLP_ST_COUNT]; /* the part of t_stage_ms recorded while the   */
  int32_t n_stage32[AHLP_ST_COUNT];   /* blocks were factored in FP32 (SYRK, FACTOR, */
                                      /* SCHUR), and its number of timed launches  */
} ahlp_ipm_result_t;

/* One interior-point iteration of the last ahlp_ipm_solve (see
 * ahlp_ipm_history). */
typedef struct {
  double mu;              /* x'z / n_tot at the top of the iteration ((x'z + s'w) /   */
                          /* (n_tot + bounded variables) with upper bounds)           */
  double sigma;           /* centring parameter (mu_aff / mu)^3 of Mehrotra's rule     */
  double alpha_p, alpha_d;/* primal and dual step lengths taken                        */
  double bkerr_pred;      /* backward error of the predictor direction after          */
                          /* refinement, on the unregularized Newton system           */
  double bkerr_corr;      /* the same for the corrector (Mehrotra's direction)        */
  int32_t refine_pred;    /* refinement corrections of the predictor                  */
  int32_t refine_corr;    /* refinement corrections of the corrector                  */
  int32_t fp32;           /* 1 if the blocks of this iteration were factored in FP32  */
  int32_t correctors;     /* Gondzio correctors kept in this iteration                */
} ahlp_ipm_iter_t;

/* Fills *opts with the defaults listed above. */
void ahlp_ipm_default_opts(ahlp_ipm_opts_t* opts);

/* Packs the problem into library-owned device memory (tile-major blocks; link
 * rows as compressed sparse rows and columns).  The caller may free desc's
 * arrays on return.  Synchronizes `stream`.  Errors: AHLP_EINVAL for sizes out
 * of range, AHLP_ENUMERIC for non-finite data, AHLP_ENOMEM, AHLP_EHIP. */
ahlp_status_t ahlp_problem_create(const ahlp_problem_desc_t* desc, hipStream_t stream,
                                  ahlp_problem_t* out);

/* Releases everything the handle owns.  NULL is accepted. */
ahlp_status_t ahlp_problem_destroy(ahlp_problem_t p);

/* Factorization, Alg. 2 of Sec. 3.2 in the normal-equation form: per block
 * M_i = A_i D_i A_i' (+ delta I) and its Cholesky factor, W_i = L_i^-1 B_i with
 * B_i = [A_i D_i F_i' | C_i], the Schur complement S = K0' - sum W_i' W_i (block
 * tridiagonal over the link pairs plus the x_0 border, App. A), and its
 * factorization.  x, z: DEVICE [n_tot], copied; must be finite and positive
 * (checked on the device; reported by the next synchronizing call as
 * AHLP_ENUMERIC).  The factors stay in the handle until the next factor call. */
ahlp_status_t ahlp_kkt_factor(ahlp_problem_t p, const double* x, const double* z,
                              const ahlp_factor_opts_t* opts, hipStream_t stream);

/* The same factorization with upper bounds inside the iteration (Sec. 3.2's
 * bounds x <= u kept as bounds): a bounded variable's slack s = u - x and dual
 * w are eliminated from the Newton system, which leaves the matrix of Sec. 2.3
 * with -Q in its (x, x) block, Q = diag(q), q = w / s (0 for a variable
 * without an upper bound), so D = (Z/X + Q + rho)^-1.  q: DEVICE [n_tot],
 * >= 0, copied.  Until the next factor call ahlp_kkt_solve (and its
 * refinement and backward error) works on
 *     [-Q A' I; A 0 0; Z 0 X] [dx; dy; dz] = [rx; ry; rz],
 * whose rx for a bounded problem is r_d + S^-1 (r_sw - W r_u) (r_u = u - x -
 * s, r_sw the (s, w) complementarity residual), with ds = r_u - dx and dw =
 * S^-1 (r_sw - W ds) recovered by the caller.  Errors as ahlp_kkt_factor;
 * the first call allocates the copy of q. */
ahlp_status_t ahlp_kkt_factor_bounded(ahlp_problem_t p, const double* x, const double* z,
                                      const double* q, const ahlp_factor_opts_t* opts,
                                      hipStream_t stream);

/* Solve, Alg. 3 of Sec. 3.2: (dx, dy, dz) for the Newton system of Sec. 2.3
 *     [0 A' I; A 0 0; Z 0 X] [dx; dy; dz] = [rx; ry; rz]
 * at the (x, z) of the last factorization.  All six vectors are DEVICE memory
 * (rx, dx, rz, dz: [n_tot]; ry, dy: [m_tot]); outputs must not alias inputs.
 * With max_refine > 0 the direction is refined in FP64 against the
 * unregularized matrix until the backward error is <= refine_tol (this
 * synchronizes the stream once per correction).  *bkerr (host, may be NULL)
 * receives the final backward error when max_refine > 0.
 * AHLP_ESTATE if no factorization exists. */
ahlp_status_t ahlp_kkt_solve(ahlp_problem_t p, const double* rx, const double* ry,
                             const double* rz, double* dx, double* dy, double* dz,
                             int32_t max_refine, double refine_tol, double* bkerr,
                             hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, results and errors as ahlp_kkt_solve, but the solve's
 * workspace (solve-phase and Schur-solve vectors, refinement residual and
 * correction, reduction partials and scalar slots) lives in the library's
 * static device array of 32 MiB per GPU (held until the process ends) instead
 * of the handle's.  The call allocates nothing.  Problems whose workspace
 * exceeds the array are refused with AHLP_EINVAL (the N = 512 workload, 256 x
 * 512 blocks, needs about 24 MiB).  Every call on one GPU shares that GPU's
 * array and clears it first: calls that overlap on one GPU (other streams,
 * other threads, other handles) race and must be ordered by the caller. */
ahlp_status_t ahlp_kkt_solve_noalloc(ahlp_problem_t p, const double* rx, const double* ry,
                                     const double* rz, double* dx, double* dy, double* dz,
                                     int32_t max_refine, double refine_tol, double* bkerr,
                                     hipStream_t stream);

/* Transposed solve with the factors of the last ahlp_kkt_factor: (wx, wy, wz)
 * with
 *     K' [wx; wy; wz] = [gx; gy; gz],   K = [0 A' I; A 0 0; Z 0 X]
 * the Newton matrix of Sec. 2.3 at the (x, z) of that factorization.  This is
 * the adjoint of the interior-point end point: with the barrier parameter
 * fixed, the KKT conditions of Sec. 2.3 define (x, y, z) as a function of
 * (b, c) whose derivative is K^-1 [dc; db; 0], so the gradient of a scalar
 * L(x, y, z) is dL/dc = wx, dL/db = wy for g = (dL/dx, dL/dy, dL/dz).  Since
 * K' = diag(I, I, Z^-1) K diag(I, I, Z), the call runs one Newton solve of
 * (gx, gy, z gz), refined as in ahlp_kkt_solve (max_refine, refine_tol, *bkerr
 * refer to that Newton system), and returns wz = dz / z.  All six vectors are
 * DEVICE memory (gx, wx, gz, wz: [n_tot]; gy, wy: [m_tot]); outputs must not
 * alias inputs.  AHLP_ESTATE if no factorization exists. */
ahlp_status_t ahlp_kkt_adjoint(ahlp_problem_t p, const double* gx, const double* gy,
                               const double* gz, double* wx, double* wy, double* wz,
                               int32_t max_refine, double refine_tol, double* bkerr,
                               hipStream_t stream);

/* Gradient of a scalar L(x*, f*) of the interior-point end point and its
 * objective f* = c'x* with respect to the LP data, by one transposed solve
 * with the factors of the last ahlp_kkt_factor (taken at the end point; the
 * derivative is the one of ahlp_kkt_adjoint, the KKT map of Sec. 2.3 with the
 * barrier parameter fixed).  With g = dL/dx* + (dL/df*) c:
 *     K' w = (g, 0, 0),   dL/db = w_y,   dL/dc = w_x + (dL/df*) x*
 * where x* is the x of that factorization.  gx: DEVICE [n_tot] (dL/dx*; NULL
 * means zero); gf: dL/df* (host value); grad_b: DEVICE [m_tot] and grad_c:
 * DEVICE [n_tot], outputs (must not alias gx).  max_refine, refine_tol and
 * *bkerr as in ahlp_kkt_adjoint.  AHLP_ESTATE if no factorization exists,
 * AHLP_EINVAL for null outputs or a non-finite gf. */
ahlp_status_t ahlp_lp_gradient(ahlp_problem_t p, const double* gx, double gf, double* grad_b,
                               double* grad_c, int32_t max_refine, double refine_tol,
                               double* bkerr, hipStream_t stream);

/* Replaces the right-hand side b and the cost c of the LP (Sec. 2.2) with new
 * DEVICE vectors b [m_tot] and c [n_tot] (copied; the matrix and the factors
 * are untouched).  Recomputes the norms the stopping test uses, so it
 * synchronizes `stream`.  Errors: AHLP_EINVAL for null pointers,
 * AHLP_ENUMERIC for non-finite entries. */
ahlp_status_t ahlp_problem_set_bc(ahlp_problem_t p, const double* b, const double* c,
                                  hipStream_t stream);

/* How the per-block stages of the factorization (SYRK, link columns, block
 * Cholesky with W_i and the Schur products; the per-block steps of Alg. 2,
 * Sec. 3.2) are launched.  Blocks of uneven size go largest first and the
 * block factor runs in two buckets, by whether the bordered block fits the
 * panel kernel.
 * AHLP_LAUNCH_BATCHED (default): one launch per stage over all blocks (the
 * SYRK, the link columns on a second stream beside it, the two factor
 * buckets).
 * AHLP_LAUNCH_PER_BLOCK: the same kernels, one launch per block and stage, in
 * block order.
 * AHLP_LAUNCH_FUSED: the panel bucket in one persistent launch over a
 * largest-first block queue, in which each CU's workgroup forms the next
 * block's link columns and SYRK while it factors the previous one; the column
 * bucket, if any, beside it with one launch per stage.
 * The arithmetic per block is the same in all three, so results are bitwise
 * equal.  Errors: AHLP_EINVAL. */
enum { AHLP_LAUNCH_BATCHED = 0, AHLP_LAUNCH_PER_BLOCK = 1, AHLP_LAUNCH_FUSED = 2 };
ahlp_status_t ahlp_problem_set_launch(ahlp_problem_t p, int32_t mode);

/* Chooses the block-factor kernel (the block factorization and the solve
 * against the linking columns of Alg. 2, Sec. 3.2) for every bordered
 * tile-row count rt that the problem's blocks have and at least two kernels
 * can hold (rt <= 40): the panel kernel with four waves per block (panel
 * accumulators in registers, rt <= 24, two workgroups per CU), the panel
 * kernel with eight waves (rt <= 40, one per CU) or the column kernel (one
 * tile column at a time through LDS, any rt).  Without tuning, the first of
 * these that fits is used.  Entries for this GPU architecture found in the
 * text file cache_path (HOST string, may be NULL) are used as they are; every
 * other rt is measured on the problem's own blocks of that rt at x = z = 1
 * (the faster of two timed launches per kernel, each after rebuilding the
 * blocks' inputs) and, with a cache_path, appended to the file as
 * "<arch> <rt> <panel|column|panel8> <us panel> <us column> <us panel8>"
 * (-1 for a kernel that cannot hold the blocks).  *measured (host, may be
 * NULL) receives the number of rt values timed.  Since buckets of different
 * kernels run side by side and share the CUs, the whole factorization is then
 * timed with these choices and with the default rule, and the faster is
 * kept for later factorizations.  Overwrites the factors (factor again
 * before solving).
 * Synchronizes `stream`.  Errors: AHLP_EINVAL (also for an unwritable cache
 * file), AHLP_EHIP. */
ahlp_status_t ahlp_autotune(ahlp_problem_t p, const char* cache_path, int32_t* measured,
                            hipStream_t stream);

/* The Mehrotra predictor-corrector loop (Sec. 2.3) around factor and solve.
 * x, z: DEVICE [n_tot], y: DEVICE [m_tot]; outputs, and inputs when
 * opts->start == 1.  Synchronous.  res (host) receives the summary.
 * Returns AHLP_OK, AHLP_WMAXITER, AHLP_WSTALL or an error. */
ahlp_status_t ahlp_ipm_solve(ahlp_problem_t p, const ahlp_ipm_opts_t* opts, double* x,
                             double* y, double* z, ahlp_ipm_result_t* res,
                             hipStream_t stream);

/* Per-iteration record of the last ahlp_ipm_solve on p (Sec. 2.3 iteration:
 * centrality, step lengths and the backward error of each Newton direction).
 * out: HOST array of cap entries (may be NULL when cap == 0); *count (host)
 * receives the number of iterations of that run, of which min(cap, *count)
 * are written.  Errors: AHLP_EINVAL for a null handle or count, cap < 0. */
ahlp_status_t ahlp_ipm_history(ahlp_problem_t p, ahlp_ipm_iter_t* out, int32_t cap,
                               int32_t* count);

/* For a problem with upper bounds (desc.ub): the slacks s = u - x and their
 * duals w at the end of the last ahlp_ipm_solve (the dual of the LP is
 * A'y + z - w = c).  s, w: DEVICE [n_tot] or NULL, zero where a variable has no
 * upper bound.  Stream ordered.  AHLP_ESTATE if the problem has no bounds. */
ahlp_status_t ahlp_ipm_bound_duals(ahlp_problem_t p, double* s, double* w, hipStream_t stream);

/* Last error message of this thread ("" when none). */
const char* ahlp_last_error(void);

/* ---- device ceilings (measurement aids, not part of the method) ----------
 * Achievable rates of this device, so that kernels can be reported against
 * measured ceilings beside the published peaks.  They synchronize `stream`
 * and allocate a small device buffer of their own. */

/* Throughput of the MFMA instruction the factorization kernels use
 * (precision AHLP_FP64: v_mfma_f64_16x16x4f64; AHLP_FP32_REFINE:
 * v_mfma_f32_16x16x4f32), on eight independent accumulators per wave, eight
 * waves per SIMD, on every CU, no memory traffic: *tflops in TFLOP/s, the
 * best of three timed launches after one untimed.  AHLP_EINVAL for another
 * precision or a null pointer. */
ahlp_status_t ahlp_ceiling_mfma(int32_t precision, double* tflops, hipStream_t stream);

/* HBM read bandwidth of a streaming pass over the DEVICE buffer buf of n
 * doubles (16-byte aligned, n >= 2; make it much larger than the caches, a
 * GiB or more), with 16-byte nontemporal loads: *gbps in GB/s (1e9 bytes),
 * the best of three timed passes after one untimed.  The contents are read,
 * never written.  AHLP_EINVAL for null or misaligned pointers or n < 2. */
ahlp_status_t ahlp_ceiling_hbm_read(const double* buf, int64_t n, double* gbps,
                                    hipStream_t stream);

/* Latency of the block factor's one-wave 16x16 tile Cholesky (FP64, the
 * elimination of the diagonal tile that sits on each block's dependency
 * chain, Alg. 2's factorization of M_i): one wave per CU factors an LDS tile
 * 256 times; *us_per_tile in microseconds, the best of three timed launches
 * after one untimed.  beside_mfma = 1 adds four waves per workgroup that
 * stream FP64 MFMAs meanwhile, one of them on the factoring wave's SIMD (as
 * a co-resident block's wave is in the factor); 0 leaves the SIMD to the
 * factoring wave.  AHLP_EINVAL for a null pointer or beside_mfma other than
 * 0 or 1. */
ahlp_status_t ahlp_ceiling_tile_chol(int32_t beside_mfma, double* us_per_tile,
                                     hipStream_t stream);

/* ---- inspection (tests and profiling; synchronize the stream) ------------
 * Copy intermediate results of the last factorization to HOST memory in the
 * canonical dense layouts below.  They exist so that every stage can be
 * compared with an independent implementation. */

/* Sizes: n_tot, m_tot, number of link rows sum(l), n0. */
ahlp_status_t ahlp_problem_sizes(ahlp_problem_t p, int64_t* n_tot, int64_t* m_tot,
                                 int64_t* n_link, int32_t* n0);

/* Block i: L (m_i x m_i, row-major, lower triangle; upper part zero) and
 * W = L^-1 B_i (m_i x k_i row-major, k_i = l_{i-1} + l_i + n0, columns ordered
 * [pair i-1 | pair i | x_0]).  Either pointer may be NULL.  FP32 factors are
 * widened to FP64. */
ahlp_status_t ahlp_debug_block(ahlp_problem_t p, int32_t i, double* L, double* W);

/* The assembled Schur complement S = K0' - sum W_i' W_i as one dense
 * (sum l + n0)^2 row-major array (small problems only), before factorization. */
ahlp_status_t ahlp_debug_schur(ahlp_problem_t p, double* S);

/* Pivots replaced by the pivot rule in the last factorization (synchronizes). */
ahlp_status_t ahlp_debug_pivots(ahlp_problem_t p, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* AHLP_H */
