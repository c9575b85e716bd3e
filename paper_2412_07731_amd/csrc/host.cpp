// Host side of libahlp: problem packing, stage orchestration on one HIP
// stream, FP64 iterative refinement and the Mehrotra predictor-corrector loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <fstream>
#include <sstream>
#include <string>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ahlp.h"
#include "common.h"
#include "kernels.h"

using namespace ahlp;

namespace {

thread_local std::string g_err;

ahlp_status_t fail(ahlp_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? AHLP_ENOMEM : AHLP_EHIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define CHK(expr)                      \
  do {                                 \
    ahlp_status_t s_ = (expr);         \
    if (s_ != AHLP_OK) return s_;      \
  } while (0)

inline long long r16(long long v) { return (v + 15) / 16 * 16; }

// Device allocation registry: everything is freed by destroy.
struct DevMem {
  std::vector<void*> ptrs;
  ~DevMem() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  ahlp_status_t alloc(T** out, long long count) {
    *out = nullptr;
    if (count <= 0) count = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)count * sizeof(T));
    if (e != hipSuccess)
      return fail(AHLP_ENOMEM, "hipMalloc of %lld bytes failed: %s", (long long)(count * sizeof(T)),
                  hipGetErrorString(e));
    ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return AHLP_OK;
  }
};

struct StageTimer {
  bool on = false;
  unsigned mask = ~0u;        // stages recorded while on (bit per AHLP_ST_*)
  hipStream_t st = nullptr;
  bool f32 = false;           // stages recorded now belong to an FP32 factorization
  struct Rec { int stage; bool f32; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<size_t> open;   // indices into pending of records not yet ended (nesting)
  std::vector<hipEvent_t> pool;
  double ms[AHLP_ST_COUNT] = {0};
  int cnt[AHLP_ST_COUNT] = {0};
  double ms32[AHLP_ST_COUNT] = {0};   // the part of ms recorded with f32 set
  int cnt32[AHLP_ST_COUNT] = {0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  bool records(int stage) const { return on && ((mask >> stage) & 1u); }
  void begin(int stage) {
    if (!on) return;
    if (!((mask >> stage) & 1u)) {   // keeps nesting balanced, records nothing
      open.push_back(SIZE_MAX);
      return;
    }
    Rec r{stage, f32, get(), get()};
    (void)hipEventRecord(r.a, st);
    open.push_back(pending.size());
    pending.push_back(r);
  }
  void end() {
    if (!on || open.empty()) return;
    if (open.back() != SIZE_MAX) (void)hipEventRecord(pending[open.back()].b, st);
    open.pop_back();
  }
  // call after a stream synchronization
  void collect() {
    open.clear();
    for (auto& r : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.stage] += t;
        cnt[r.stage] += 1;
        if (r.f32) {
          ms32[r.stage] += t;
          cnt32[r.stage] += 1;
        }
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    collect();
    for (int i = 0; i < AHLP_ST_COUNT; ++i) { ms[i] = 0; cnt[i] = 0; ms32[i] = 0; cnt32[i] = 0; }
  }
  ~StageTimer() {
    for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

// Block-factor kernels (bf_kernel entries): the four-wave panel kernel, the
// column-at-a-time kernel, the eight-wave panel kernel.
enum { BFK_PANEL = 0, BFK_COLUMN = 1, BFK_PANEL8 = 2 };

// Segments of an interior-point iteration between host synchronizations:
// A = factorization + predictor (+ check, step lengths, mu_aff), B = corrector
// (+ check, step lengths), per factor precision; C = step + next residuals.
enum { SEG_A64 = 0, SEG_A32, SEG_B64, SEG_B32, SEG_C, SEG_COUNT };
// What a captured segment bakes in besides the problem's own buffers.
// launch_gen counts changes of the launch configuration (block-factor
// buckets and order, launch mode), which a captured segment also bakes in.
struct SegKey {
  const double *x, *y, *z;
  double rho, delta, eta;
  unsigned launch_gen;
  bool operator==(const SegKey& o) const {
    return x == o.x && y == o.y && z == o.z && rho == o.rho && delta == o.delta &&
           eta == o.eta && launch_gen == o.launch_gen;
  }
};

// Device workspace of one refined Newton solve (Alg. 3 with the refinement
// loop): the solve-phase vectors, the Schur-solve vectors of either Schur
// path, the refinement residual and correction, the reduction partials and
// the scalar slots.
struct SolveWs {
  double *rhx, *vx, *tv, *qn, *s, *w, *u, *dyp, *g, *part, *segrhs, *xp;
  double *br, *bw, *bup, *bpb, *bu0p;
  double *ex, *ey, *ez, *cx, *cy, *cz, *gc;
  double *red_part, *scal;
};

struct ahlp_problem_s {
  int device = 0;
  int N = 0, n0 = 0, n0p = 0, P = 0, G = 0;
  int ng = 0, nb = 0;   // global rows; width of the Schur border (ng + n0)
  std::vector<int> m, n, l;
  std::vector<BlockInfo> hb;
  std::vector<long long> loff, tdoff, tooff, eoff, zoff, suboff;
  std::vector<int2> seg;
  long long n_tot = 0, m_tot = 0, nl = 0, mblk = 0, x0off = 0, d0off = 0, dp_total = 0;
  long long nle = 0;    // link rows plus global rows: the dual rows after the blocks
  long long f0first = 0;   // first row of F0 that may be nonzero (nl when only Wg0 is)
  long long vp_total = 0, q_total = 0, a_total = 0, c_total = 0, lb_total = 0, linv_total = 0,
            pq_total = 0;
  int max_rt = 0, lmax = 0, max_kt = 0;
  double colabs1_max = 1.0, rowabs_max = 0.0, b_inf = 0.0, c_inf = 0.0;
  DevMem mem;

  // problem data
  BlockInfo* blk = nullptr;
  // F0: the x_0 coupling of the dual rows after the blocks, (nl + ng) x n0:
  // the link rows' F0, then the global rows' Wg0 (null when all zero)
  double *A = nullptr, *C = nullptr, *F0 = nullptr, *b = nullptr, *c = nullptr;
  float* A32 = nullptr;
  int *lptr = nullptr, *lcol = nullptr, *cptr = nullptr, *crow = nullptr;
  double *lval = nullptr, *cval = nullptr;
  // the global rows as compressed rows over the padded x (index dpoff + column)
  int *gptr = nullptr, *gidx = nullptr;
  double* gval = nullptr;
  int4* syrk_items = nullptr;
  int nsyrk = 0;
  // block-factor buckets: bf_order[0, n_panel) for the four-wave panel
  // kernel, then n_panel8 blocks for the eight-wave one, then n_col blocks
  // for the column kernel, each largest first
  int* bf_order = nullptr;
  int n_panel = 0, n_panel8 = 0, n_col = 0, rt_panel = 0, rt_panel8 = 0, rt_col = 0;
  // per-block launch mode (the reference the batched launches are compared
  // with): block i's SYRK items, link items, and its index in an identity list
  int launch_mode = AHLP_LAUNCH_BATCHED;
  int num_cu = 1;
  int* fused_queue = nullptr;          // the fused launch's block queue counter
  // host copies of the work lists and the column-kernel bucket's own SYRK and
  // link items (the fused launch covers the panel bucket)
  std::vector<int4> h_syrk;
  std::vector<int2> h_link;
  std::vector<int> h_bf;
  int4* col_syrk_items = nullptr;
  int2* col_link_items = nullptr;
  int ncol_syrk = 0, ncol_link = 0;
  unsigned launch_gen = 0;   // bumped whenever bf_order, the buckets or launch_mode change
  // block-factor kernel per bordered tile-row count (0 panel, 1 column; the
  // default rule is panel wherever it fits); set by ahlp_autotune
  std::vector<int> bf_kernel;
  std::vector<int> syrk_off, syrk_cnt, link_off, link_cnt;
  int* ident = nullptr;
  int2* link_items = nullptr;
  int nlink = 0;
  int2 *rowtiles = nullptr, *coltiles = nullptr, *c0tiles = nullptr;
  int nrt = 0, nct = 0, nc0 = 0;
  int* d_l = nullptr;
  long long *d_loff = nullptr, *d_tdoff = nullptr, *d_tooff = nullptr, *d_eoff = nullptr,
            *d_zoff = nullptr, *d_suboff = nullptr;
  int2* d_seg = nullptr;

  // factorization
  double *Dp = nullptr, *xs = nullptr, *zs = nullptr;
  double *LB = nullptr, *LINV = nullptr, *PQ = nullptr;
  float *LB32 = nullptr, *LINV32 = nullptr;
  double *Td = nullptr, *To = nullptr, *E = nullptr, *S00 = nullptr, *thrT = nullptr;
  double *CL = nullptr, *CLi = nullptr, *CYn = nullptr, *CZ = nullptr, *CG = nullptr,
         *CSub = nullptr, *Lb = nullptr, *Lbi = nullptr, *S00w = nullptr, *segout = nullptr;
  // tile path of the Schur factorization (pairs <= 32 rows, border <= 64)
  bool fast = false;          // Schur factor by cyclic reduction (else the segmented chain)
  int tp = 0;                 // its tiles per pair side
  int t0 = 0, s00_chunk = 16, s00_parts = 0;
  double *BD = nullptr, *BC = nullptr, *BEt = nullptr, *FLi = nullptr, *FXL = nullptr,
         *FXR = nullptr, *FGt = nullptr, *FLb = nullptr, *FLbi = nullptr, *s00part = nullptr;
  DevInfo* info = nullptr;   // lives in the last slot of the handle's own ws.scal
  bool factored = false;
  int fprec = AHLP_FP64;
  double rho = 0, delta = 0;
  int pivots_seen = 0;

  // workspace of a refined solve (allocated at create; ahlp_kkt_solve_noalloc
  // points it into the library's static device array for one call)
  SolveWs ws{};
  double *aty = nullptr, *gdir = nullptr;
  double *ones = nullptr, *zerosn = nullptr;
  // predictor/corrector right-hand sides by linearity (padded v-space) and scaled vectors
  double *ta = nullptr, *aw1 = nullptr, *aw2 = nullptr, *tc = nullptr, *w1p = nullptr,
         *w2p = nullptr;
  double* adj_rz = nullptr;   // z g_z of the transposed solve
  double *grad_g = nullptr, *grad_wz = nullptr;   // ahlp_lp_gradient: its right-hand side, w_z
  // upper bounds inside the iteration (allocated when some are finite): ub
  // (+inf where none) and ufin (u or 0); the interior-point run's slacks s,
  // duals w, their directions (predictor ds, dw and corrector), r_u = u - x -
  // s, q = w/s, zw = z - w, the reduced x right-hand sides of predictor and
  // corrector, and minima helpers of the start
  long long nU = 0;
  double ub_inf = 0.0;
  double *ub = nullptr, *ufin = nullptr, *bs = nullptr, *bw = nullptr, *bdsa = nullptr,
         *bdwa = nullptr, *bds = nullptr, *bdw = nullptr, *bru = nullptr, *bq = nullptr,
         *bzw = nullptr, *brdt = nullptr, *brxc = nullptr, *bsm = nullptr, *bwm = nullptr,
         *bqapi = nullptr;
  const double* qcur = nullptr;   // q of the current factorization (nullptr: none)
  // Gondzio correctors: right-hand side, candidate direction, zero y-vector
  double *g_r = nullptr, *g_dx = nullptr, *g_dy = nullptr, *g_dz = nullptr, *zerosm = nullptr;
  double *rp = nullptr, *rd = nullptr, *rzv = nullptr, *dxa = nullptr, *dya = nullptr,
         *dza = nullptr, *dx = nullptr, *dy = nullptr, *dz = nullptr;
  double* h_scal = nullptr;   // pinned host mirror of ws.scal
  // side stream (default priority) for the link-column gather, which runs
  // beside the block SYRK: event fork from the caller's stream, join before
  // the block factor
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // graph mode of ahlp_ipm_solve: the solve runs on gstream (capturable; event
  // fork/join with the caller's stream) and the three host-sync-free segments
  // of an iteration are replays of captured graphs (see run_segment)
  hipStream_t gstream = nullptr;
  hipEvent_t ev_gin = nullptr, ev_gout = nullptr;
  bool use_graph = false;
  struct SegGraph {
    hipGraphExec_t exec = nullptr;
    SegKey key{};
  } graphs[SEG_COUNT];
  StageTimer timer;
  std::vector<ahlp_ipm_iter_t> hist;   // per-iteration record of the last interior-point run
  double rows_bytes = 0.0;      // algorithmic bytes of the timed row passes
  double a_bytes = 0, c_bytes = 0, xv_bytes = 0, x0_bytes = 0, yv_bytes = 0;

  // host-side handles (device buffers are released by mem); also runs when
  // creation fails part way
  ~ahlp_problem_s() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (ev_gin) (void)hipEventDestroy(ev_gin);
    if (ev_gout) (void)hipEventDestroy(ev_gout);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (h_scal) (void)hipHostFree(h_scal);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace {

constexpr int NSCAL = 32;
// scal slots: 0-5 residual stage, 9 |K| norm, 10-12 step lengths and mu_aff,
// 20-28 refinement check (|r|, |e|, |d| per block row), 31 device info
constexpr int S_AP = 10, S_AD = 11, S_MUAFF = 12, S_SMU = 13, S_GP = 14, S_GD = 15, S_RN = 20,
              S_EN = 23, S_DN = 26;
// with upper bounds: s'w, |r_u|_inf, u'w, (s + a_p ds)'(w + a_d dw) and max q
constexpr int S_SW = 6, S_RU = 7, S_UW = 16, S_MUAFF_SW = 17, S_QMAX = 18;
static_assert(sizeof(DevInfo) <= sizeof(double), "device info must fit one scal slot");

ahlp_status_t check_info(ahlp_problem_t p, hipStream_t st, bool* nonfinite) {
  DevInfo h{};
  HIPCHK(hipMemcpyAsync(&h, p->info, sizeof h, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  p->pivots_seen = h.pivots;
  if (h.nonfinite & 2)
    return fail(AHLP_EHIP, "the fused factorization launch gave up waiting for its own stages");
  if (nonfinite) *nonfinite = h.nonfinite != 0;
  return AHLP_OK;
}

// Places the workspace of one refined solve at base (256-byte aligned
// pieces, each at least one element) and returns its size in bytes; with
// base == nullptr only the size.  The handle's own workspace and the static
// one of ahlp_kkt_solve_noalloc use this one layout.
size_t solve_ws_layout(const ahlp_problem_s* p, double* base, SolveWs* ws) {
  size_t off = 0;   // bytes
  auto take = [&](double** dst, long long count) {
    if (count < 1) count = 1;
    if (base && ws) *dst = reinterpret_cast<double*>(reinterpret_cast<char*>(base) + off);
    off += ((size_t)count * sizeof(double) + 255) / 256 * 256;
  };
  SolveWs tmp{};
  SolveWs& w = ws ? *ws : tmp;
  const long long n = p->n_tot, m = p->m_tot, nb = p->nl + p->nb;
  take(&w.rhx, n); take(&w.vx, p->dp_total); take(&w.xp, p->dp_total);
  take(&w.tv, p->vp_total); take(&w.dyp, p->vp_total); take(&w.qn, p->q_total);
  take(&w.s, nb); take(&w.w, nb); take(&w.u, nb);
  take(&w.g, n); take(&w.part, (long long)p->N * std::max(p->n0, 1));
  take(&w.segrhs, (long long)std::max(p->G, 1) * SEGRHS_STRIDE);
  take(&w.ex, n); take(&w.ey, m); take(&w.ez, n);
  take(&w.cx, n); take(&w.cy, m); take(&w.cz, n); take(&w.gc, n);
  take(&w.red_part, (long long)MAXRED * RED_PARTIALS); take(&w.scal, NSCAL);
  if (p->fast) {
    const long long Pt = std::max(p->P, 1), T0 = std::max(p->t0, 1), tp = p->tp;
    take(&w.br, Pt * tp * 16); take(&w.bw, Pt * tp * 16); take(&w.bup, Pt * tp * 16);
    take(&w.bpb, Pt * T0 * 16); take(&w.bu0p, T0 * 16);
  }
  return off;
}

// ------------------------------------------------------------- factor
// Block-factor kernel for bordered tile-row count rt: the autotuned choice
// (bf_kernel) or the default rule, the four-wave panel kernel where it fits,
// else the eight-wave one, else the column kernel.
int bf_choice(const ahlp_problem_s* p, int rt) {
  const int k = rt < (int)p->bf_kernel.size() ? p->bf_kernel[rt] : -1;
  if (k == BFK_PANEL && block_factor_panel_fits(rt)) return BFK_PANEL;
  if (k == BFK_PANEL8 && block_factor_panel8_fits(rt)) return BFK_PANEL8;
  if (k == BFK_COLUMN) return BFK_COLUMN;
  if (block_factor_panel_fits(rt)) return BFK_PANEL;
  if (block_factor_panel8_fits(rt)) return BFK_PANEL8;
  return BFK_COLUMN;
}

// Block-factor buckets: blocks largest first (rt, then mt, then nt), the
// four-wave panel bucket, the eight-wave panel bucket, the column bucket;
// sets n_* and rt_* of each.
std::vector<int> bf_buckets(ahlp_problem_t p) {
  const int N = p->N;
  std::vector<int> bysize(N);
  for (int i = 0; i < N; ++i) bysize[i] = i;
  std::stable_sort(bysize.begin(), bysize.end(), [&](int a, int c) {
    const BlockInfo &x = p->hb[a], &y = p->hb[c];
    if (x.rt != y.rt) return x.rt > y.rt;
    if (x.mt != y.mt) return x.mt > y.mt;
    return x.nt > y.nt;
  });
  std::vector<int> out;
  int* cnt[3] = {&p->n_panel, &p->n_col, &p->n_panel8};
  int* rtm[3] = {&p->rt_panel, &p->rt_col, &p->rt_panel8};
  for (int k : {BFK_PANEL, BFK_PANEL8, BFK_COLUMN}) {
    *cnt[k] = 0;
    *rtm[k] = 0;
    for (int i : bysize)
      if (bf_choice(p, p->hb[i].rt) == k) {
        out.push_back(i);
        ++*cnt[k];
        *rtm[k] = std::max(*rtm[k], p->hb[i].rt);
      }
  }
  return out;
}

// Block-factor buckets into p->h_bf and bf_order, and the column bucket's
// own SYRK and link items (the fused launch covers the panel bucket); every
// captured graph holds the old ones, so the launch generation moves on.
ahlp_status_t set_buckets(ahlp_problem_t p, hipStream_t st) {
  p->h_bf = bf_buckets(p);
  std::vector<int4> cs;
  std::vector<int2> cl;
  for (int k = p->n_panel; k < p->N; ++k) {
    const int i = p->h_bf[k];
    cs.insert(cs.end(), p->h_syrk.begin() + p->syrk_off[i],
              p->h_syrk.begin() + p->syrk_off[i] + p->syrk_cnt[i]);
    cl.insert(cl.end(), p->h_link.begin() + p->link_off[i],
              p->h_link.begin() + p->link_off[i] + p->link_cnt[i]);
  }
  p->ncol_syrk = (int)cs.size();
  p->ncol_link = (int)cl.size();
  HIPCHK(hipMemcpyAsync(p->bf_order, p->h_bf.data(), sizeof(int) * p->h_bf.size(),
                        hipMemcpyHostToDevice, st));
  if (!cs.empty())
    HIPCHK(hipMemcpyAsync(p->col_syrk_items, cs.data(), sizeof(int4) * cs.size(),
                          hipMemcpyHostToDevice, st));
  if (!cl.empty())
    HIPCHK(hipMemcpyAsync(p->col_link_items, cl.data(), sizeof(int2) * cl.size(),
                          hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));   // the host vectors are temporaries
  ++p->launch_gen;
  return AHLP_OK;
}

// The same kernels, one launch per block and stage, in block order on st:
// the reference for the batched launches (identical arithmetic per block).
template <typename T>
ahlp_status_t factor_blocks_per_block(ahlp_problem_t p, hipStream_t st, T* LB, T* LINV,
                                      const T* A) {
  p->timer.begin(AHLP_ST_SYRK);
  for (int i = 0; i < p->N; ++i) {
    launch_link<T>(st, p->blk, p->link_items + p->link_off[i], p->link_cnt[i], p->nb, p->A, p->C,
                   p->lptr, p->lcol, p->lval, p->Dp, LB, p->PQ);
    launch_syrk<T>(st, p->blk, p->syrk_items + p->syrk_off[i], p->syrk_cnt[i], A, p->Dp, LB,
                   p->delta);
  }
  p->timer.end();
  p->timer.begin(AHLP_ST_FACTOR);
  for (int i = 0; i < p->N; ++i) {
    const int rt = p->hb[i].rt, k = bf_choice(p, rt);
    if (k == BFK_COLUMN)
      launch_block_factor_col<T>(st, p->blk, p->ident + i, 1, rt, LB, LINV, p->PQ, p->info);
    else
      launch_block_factor_panel<T>(st, p->blk, p->ident + i, 1, rt, LB, LINV, p->PQ, p->info,
                                   k == BFK_PANEL8 ? 8 : 4, p->max_kt);
  }
  p->timer.end();
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

// The four-wave panel bucket fused (link columns, SYRK, block factor and
// Schur contributions in one persistent launch); the other buckets, if any,
// run their own link, SYRK and factor launches on the side stream beside it.
template <typename T>
ahlp_status_t factor_blocks_fused(ahlp_problem_t p, hipStream_t st, T* LB, T* LINV,
                                  const T* A) {
  p->timer.begin(AHLP_ST_FACTOR);
  const bool rest = p->n_panel8 + p->n_col > 0;
  if (rest) {
    HIPCHK(hipEventRecord(p->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    launch_link<T>(p->side, p->blk, p->col_link_items, p->ncol_link, p->nb, p->A, p->C, p->lptr,
                   p->lcol, p->lval, p->Dp, LB, p->PQ);
    launch_syrk<T>(p->side, p->blk, p->col_syrk_items, p->ncol_syrk, A, p->Dp, LB, p->delta);
    launch_block_factor_panel<T>(p->side, p->blk, p->bf_order + p->n_panel, p->n_panel8,
                                 p->rt_panel8, LB, LINV, p->PQ, p->info, 8, p->max_kt);
    launch_block_factor_col<T>(p->side, p->blk, p->bf_order + p->n_panel + p->n_panel8, p->n_col,
                               p->rt_col, LB, LINV, p->PQ, p->info);
    HIPCHK(hipEventRecord(p->ev_join, p->side));
  }
  launch_factor_fused<T>(st, p->blk, p->bf_order, p->n_panel, p->rt_panel, p->fused_queue, p->nb,
                         A, p->A, p->C, p->lptr, p->lcol, p->lval, p->Dp, LB, LINV, p->PQ,
                         p->delta, p->info, p->num_cu);
  if (rest) HIPCHK(hipStreamWaitEvent(st, p->ev_join, 0));
  p->timer.end();
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

template <typename T>
ahlp_status_t factor_blocks(ahlp_problem_t p, hipStream_t st, T* LB, T* LINV, const T* A) {
  if (p->launch_mode == AHLP_LAUNCH_PER_BLOCK) return factor_blocks_per_block<T>(p, st, LB, LINV, A);
  if (p->launch_mode == AHLP_LAUNCH_FUSED) return factor_blocks_fused<T>(p, st, LB, LINV, A);
  // the link gather (HBM-bound) runs on the side stream while the SYRK
  // (MFMA-bound) runs on st; they write disjoint tiles of LB
  HIPCHK(hipEventRecord(p->ev_fork, st));
  HIPCHK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
  launch_link<T>(p->side, p->blk, p->link_items, p->nlink, p->nb, p->A, p->C, p->lptr, p->lcol,
                 p->lval, p->Dp, LB, p->PQ);
  HIPCHK(hipEventRecord(p->ev_join, p->side));
  p->timer.begin(AHLP_ST_SYRK);
  launch_syrk<T>(st, p->blk, p->syrk_items, p->nsyrk, A, p->Dp, LB, p->delta);
  p->timer.end();
  p->timer.begin(AHLP_ST_FACTOR);
  HIPCHK(hipStreamWaitEvent(st, p->ev_join, 0));
  const int nb8 = p->n_panel8, nbc = p->n_col;
  const int* o8 = p->bf_order + p->n_panel;
  const int* oc = o8 + nb8;
  if (p->n_panel > 0 && nb8 + nbc > 0) {
    // the eight-wave panel and the column buckets beside the four-wave one
    HIPCHK(hipEventRecord(p->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    launch_block_factor_panel<T>(p->side, p->blk, o8, nb8, p->rt_panel8, LB, LINV, p->PQ, p->info, 8,
                                 p->max_kt);
    launch_block_factor_col<T>(p->side, p->blk, oc, nbc, p->rt_col, LB, LINV, p->PQ, p->info);
    HIPCHK(hipEventRecord(p->ev_join, p->side));
    launch_block_factor_panel<T>(st, p->blk, p->bf_order, p->n_panel, p->rt_panel, LB, LINV, p->PQ,
                                 p->info, 4, p->max_kt);
    HIPCHK(hipStreamWaitEvent(st, p->ev_join, 0));
  } else {
    launch_block_factor_panel<T>(st, p->blk, p->bf_order, p->n_panel, p->rt_panel, LB, LINV, p->PQ,
                                 p->info, 4, p->max_kt);
    launch_block_factor_panel<T>(st, p->blk, o8, nb8, p->rt_panel8, LB, LINV, p->PQ, p->info, 8,
                                 p->max_kt);
    launch_block_factor_col<T>(st, p->blk, oc, nbc, p->rt_col, LB, LINV, p->PQ, p->info);
  }
  p->timer.end();
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

ChainArgs chain_args(ahlp_problem_t p) {
  ChainArgs c{};
  c.P = p->P; c.G = p->G; c.n0 = p->nb; c.ng = p->ng;
  c.l = p->d_l; c.tdoff = p->d_tdoff; c.tooff = p->d_tooff; c.eoff = p->d_eoff;
  c.zoff = p->d_zoff; c.suboff = p->d_suboff; c.seg = p->d_seg;
  c.Td = p->Td; c.To = p->To; c.E = p->E; c.S00 = p->S00; c.thrT = p->thrT;
  c.CL = p->CL; c.CLi = p->CLi; c.CYn = p->CYn; c.CZ = p->CZ; c.CG = p->CG; c.CSub = p->CSub;
  c.Lb = p->Lb; c.Lbi = p->Lbi; c.S00w = p->S00w; c.segout = p->segout;
  c.lmax = std::max(p->lmax, 1);
  c.info = p->info;
  return c;
}

BcrArgs bcr_args(ahlp_problem_t p) {
  BcrArgs c{};
  c.P = p->P; c.n0 = p->nb; c.ng = p->ng; c.t0 = p->t0; c.tp = p->tp;
  c.l = p->d_l; c.tdoff = p->d_tdoff; c.tooff = p->d_tooff; c.eoff = p->d_eoff;
  c.Td = p->Td; c.To = p->To; c.E = p->E; c.S00 = p->S00; c.thrT = p->thrT;
  c.BD = p->BD; c.BC = p->BC; c.BEt = p->BEt;
  c.FLi = p->FLi; c.FXL = p->FXL; c.FXR = p->FXR; c.FGt = p->FGt;
  c.FLb = p->FLb; c.FLbi = p->FLbi; c.s00part = p->s00part;
  c.info = p->info;
  return c;
}

ahlp_status_t ensure_fp32(ahlp_problem_t p, hipStream_t st) {
  if (!p->A32) {
    CHK(p->mem.alloc(&p->A32, p->a_total));
    launch_convert_f32(st, p->a_total, p->A, p->A32);
  }
  if (!p->LB32) CHK(p->mem.alloc(&p->LB32, p->lb_total));
  if (!p->LINV32) CHK(p->mem.alloc(&p->LINV32, p->linv_total));
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

// D-scaling of (x, z) and the info reset (a1); the factor assumes it ran.
ahlp_status_t prep_scaling(ahlp_problem_t p, const double* x, const double* z, double rho,
                           hipStream_t st) {
  static_assert(sizeof(DevInfo) <= sizeof(double), "DevInfo lives in one scalar slot");
  launch_fill(st, 1, 0.0, reinterpret_cast<double*>(p->info));   // a kernel, not a memset: capturable
  p->timer.begin(AHLP_ST_PREP);
  launch_prep(st, p->blk, p->N, p->n0, p->x0off, p->d0off, x, z, p->qcur, rho, p->Dp, p->xs, p->zs,
              p->info);
  p->timer.end();
  return AHLP_OK;
}

// prepped: prep_scaling already ran for this (x, z, rho)
ahlp_status_t do_factor(ahlp_problem_t p, const double* x, const double* z, int prec, double rho,
                        double delta, hipStream_t st, bool prepped = false) {
  p->rho = rho;
  p->delta = delta;
  p->fprec = prec;
  if (!prepped) CHK(prep_scaling(p, x, z, rho, st));
  p->timer.f32 = prec == AHLP_FP32_REFINE;
  if (prec == AHLP_FP32_REFINE) {
    CHK(ensure_fp32(p, st));
    CHK(factor_blocks<float>(p, st, p->LB32, p->LINV32, p->A32));
  } else {
    CHK(factor_blocks<double>(p, st, p->LB, p->LINV, p->A));
  }
  p->timer.begin(AHLP_ST_SCHUR);
  launch_assemble(st, p->blk, p->N, p->nb, p->n0, p->nl, p->d_l, p->d_tdoff, p->d_tooff,
                  p->d_eoff, p->PQ, p->f0first == 0 ? p->F0 : nullptr, p->F0, p->d_loff, delta,
                  p->Dp + p->d0off, p->Td, p->To, p->E,
                  p->S00, p->thrT);
  p->timer.end();
  p->timer.f32 = false;
  p->timer.begin(AHLP_ST_TFACTOR);
  if (p->fast) launch_bcr_factor(st, bcr_args(p), p->s00_parts, p->s00_chunk);
  else launch_chain_factor(st, chain_args(p));
  p->timer.end();
  HIPCHK(hipGetLastError());
  p->factored = true;
  return AHLP_OK;
}

// Runs fn on st: directly, or in graph mode as a replay of its captured graph
// (captured on first use and whenever the key changes).  fn must launch work
// on st only (forks to the side stream join back), without host
// synchronization, allocation or memset; the kernels and arguments it records
// are then the same on every replay, so a replay equals a direct run.
template <typename F>
ahlp_status_t run_segment(ahlp_problem_t p, int id, const SegKey& key, hipStream_t st, F&& fn) {
  if (!p->use_graph) return fn();
  auto& g = p->graphs[id];
  if (!g.exec || !(g.key == key)) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    const ahlp_status_t s = fn();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != AHLP_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(AHLP_EHIP, "graph capture: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(AHLP_EHIP, "graph instantiation: %s", hipGetErrorString(ei));
    g.key = key;
  }
  HIPCHK(hipGraphLaunch(g.exec, st));
  return AHLP_OK;
}

// ------------------------------------------------------------- solve
// One pass of Alg. 3 (no refinement).  Also leaves g = A' dy in p->ws.g.
template <typename T>
void solve_blocks_fwd(ahlp_problem_t p, hipStream_t st, const T* LB, const T* LINV,
                      const double* tin) {
  launch_block_fwd<T>(st, p->blk, p->N, p->max_rt, LB, LINV, tin, p->ws.tv, p->ws.qn);
}
template <typename T>
void solve_blocks_bwd(ahlp_problem_t p, hipStream_t st, const T* LB, const T* LINV, double* dy) {
  launch_block_bwd<T>(st, p->blk, p->N, p->nb, p->nl, p->max_rt, LB, LINV, p->ws.tv, p->ws.u, dy,
                      p->ws.dyp);
}

// The dual rows after the blocks: out = base + alpha (F xp [+ F0 x0]) for the
// link rows and the global rows (out and base point at the first link row;
// x0 and the x_0 coupling only when x0 is given).
void link_global_rows(ahlp_problem_t p, const double* xp, const double* x0, const double* base,
                      double alpha, double* out, hipStream_t st) {
  const double* F0 = x0 ? p->F0 : nullptr;
  launch_linkrows(st, p->blk, p->P, p->ng, p->n0, p->d_l, p->d_loff, p->nl, p->lptr, p->lcol,
                  p->lval, p->gptr, p->gidx, p->gval, xp, x0, F0, p->f0first == 0 ? F0 : nullptr,
                  base, alpha, out);
}

// A row pass (AHLP_ST_AROWS) with its algorithmic bytes: the A tiles, the C
// tiles if any vector takes the x_0 columns, each vector, each base read and
// each output written (real sizes, not the tile padding).
void rows_pass(ahlp_problem_t p, const RowsArgs& ra, hipStream_t st) {
  p->timer.begin(AHLP_ST_AROWS);
  launch_rows_multi(st, p->blk, p->rowtiles, p->nrt, p->A, p->C, p->d0off, ra);
  p->timer.end();
  if (p->timer.records(AHLP_ST_AROWS)) {
    bool anyC = false;
    double b = p->a_bytes;
    for (int k = 0; k < ra.nv; ++k) {
      anyC = anyC || ra.with_C[k];
      b += p->xv_bytes + (ra.with_C[k] ? p->x0_bytes : 0.0) + p->yv_bytes;
      if (ra.base[k] && !ra.chain[k]) b += p->yv_bytes;
    }
    if (anyC) b += p->c_bytes;
    p->rows_bytes += b;
  }
}
void rows_pass1(ahlp_problem_t p, const double* v, const double* base, double alpha, int with_C,
                int padded, double* out, hipStream_t st) {
  RowsArgs ra{};
  ra.nv = 1;
  ra.v[0] = v; ra.base[0] = base; ra.alpha[0] = alpha; ra.out[0] = out;
  ra.with_C[0] = with_C; ra.padded[0] = padded;
  rows_pass(p, ra, st);
}

// tpre: precomputed t = r_y + A D rhx (padded v-space) or null; gout receives
// g = A' dy (default p->ws.g).
ahlp_status_t solve_once(ahlp_problem_t p, const double* rx, const double* ry, const double* rz,
                         double* dx, double* dy, double* dz, hipStream_t st,
                         const double* tpre = nullptr, double* gout = nullptr) {
  if (!gout) gout = p->ws.g;
  const bool f32 = p->fprec == AHLP_FP32_REFINE;
  p->timer.begin(AHLP_ST_SOLVE);
  launch_rhx(st, p->blk, p->N, p->n0, p->x0off, p->d0off, rx, rz, p->xs, p->Dp, p->ws.rhx, p->ws.vx);
  // t_i = ry_i + A_i D_i rhx_i (padded), s_L = ry_L + F D rhx
  if (!tpre) {
    rows_pass1(p, p->ws.vx, ry, 1.0, 0, 1, p->ws.tv, st);
    tpre = p->ws.tv;
  }
  link_global_rows(p, p->ws.vx, nullptr, ry + p->mblk, 1.0, p->ws.s, st);
  if (f32) solve_blocks_fwd<float>(p, st, p->LB32, p->LINV32, tpre);
  else solve_blocks_fwd<double>(p, st, p->LB, p->LINV, tpre);
  launch_schur_rhs(st, p->blk, p->N, p->nb, p->d_l, p->d_loff, p->nl, p->ws.qn, p->ws.rhx + p->x0off,
                   p->ws.s);
  if (p->fast) {
    BcrSolveArgs a{};
    a.c = bcr_args(p);
    a.loff = p->d_loff; a.nl = p->nl; a.s = p->ws.s; a.u = p->ws.u;
    a.r = p->ws.br; a.w = p->ws.bw; a.up = p->ws.bup; a.pb = p->ws.bpb; a.u0p = p->ws.bu0p;
    launch_bcr_solve(st, a);
  } else {
    ChainSolveArgs a{};
    a.c = chain_args(p);
    a.loff = p->d_loff; a.nl = p->nl; a.s = p->ws.s; a.w = p->ws.w; a.u = p->ws.u; a.segrhs = p->ws.segrhs;
    launch_chain_solve(st, a);
  }
  if (f32) solve_blocks_bwd<float>(p, st, p->LB32, p->LINV32, dy);
  else solve_blocks_bwd<double>(p, st, p->LB, p->LINV, dy);
  // dx_i = D_i (A_i' dy_i + F_i' dy_L - rhx_i), dz = (rz - Z dx) / X;  g = A' dy
  const DzArgs dzv{rz, p->zs, p->xs, dz};
  launch_cols(st, p->blk, p->coltiles, p->nct, p->A, p->ws.dyp, p->ws.u, p->cptr, p->crow, p->cval, 2,
              p->ws.rhx, nullptr, p->Dp, gout, dx, dzv);
  launch_ccols(st, p->blk, p->c0tiles, p->nc0, p->n0, p->C, p->ws.dyp, p->ws.part);
  launch_solve_tail(st, p->N, p->n0, p->nle, p->f0first, p->ws.part, p->F0, p->ws.u, p->x0off, p->mblk, gout, dx, dzv,
                    dy);
  p->timer.end();
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

// g = A' y (canonical), using the padded copy of the block rows.
void apply_At(ahlp_problem_t p, const double* y, int mode, const double* cvec,
              const double* zvec, double* out, hipStream_t st) {
  launch_pad_y(st, p->blk, p->N, y, p->ws.dyp);
  launch_cols(st, p->blk, p->coltiles, p->nct, p->A, p->ws.dyp, y + p->mblk, p->cptr, p->crow,
              p->cval, mode, cvec, zvec, p->Dp, mode == 0 ? out : nullptr,
              mode == 0 ? nullptr : out);
  launch_ccols(st, p->blk, p->c0tiles, p->nc0, p->n0, p->C, p->ws.dyp, p->ws.part);
  launch_x0_sum(st, p->N, p->n0, p->nle, p->f0first, p->ws.part, p->F0, y + p->mblk, mode, cvec, zvec, p->x0off,
                mode == 0 ? out : nullptr, mode == 0 ? nullptr : out);
}

// rd = cvec - A'y - zvec, and g = A'y kept in gout (one column pass)
void apply_At_both(ahlp_problem_t p, const double* y, const double* cvec, const double* zvec,
                   double* rd, double* gout, hipStream_t st) {
  launch_pad_y(st, p->blk, p->N, y, p->ws.dyp);
  launch_cols(st, p->blk, p->coltiles, p->nct, p->A, p->ws.dyp, y + p->mblk, p->cptr, p->crow,
              p->cval, 1, cvec, zvec, p->Dp, gout, rd);
  launch_ccols(st, p->blk, p->c0tiles, p->nc0, p->n0, p->C, p->ws.dyp, p->ws.part);
  launch_x0_sum(st, p->N, p->n0, p->nle, p->f0first, p->ws.part, p->F0, y + p->mblk, 1, cvec, zvec, p->x0off,
                gout, rd);
}

// out = base + alpha * A x (canonical)
void apply_A(ahlp_problem_t p, const double* x, const double* base, double alpha, double* out,
             hipStream_t st) {
  launch_pad_x(st, p->blk, p->N, p->n0, p->x0off, p->d0off, x, p->ws.xp, nullptr);
  rows_pass1(p, p->ws.xp, base, alpha, 1, 0, out, st);
  link_global_rows(p, p->ws.xp, p->ws.xp + p->d0off, base ? base + p->mblk : nullptr, alpha,
                   out + p->mblk, st);
}

ahlp_status_t read_scal(ahlp_problem_t p, int count, hipStream_t st) {
  (void)count;   // the whole slot array (incl. the device info) is copied
  HIPCHK(hipMemcpyAsync(p->h_scal, p->ws.scal, sizeof(double) * NSCAL, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  p->timer.collect();
  return AHLP_OK;
}

void red(ahlp_problem_t p, int op, long long n, const double* a, const double* b, int slot,
         hipStream_t st, const double* c = nullptr, const double* d = nullptr, double s1 = 0,
         double s2 = 0) {
  launch_reduce(st, op, n, a, b, c, d, s1, s2, p->ws.red_part, p->ws.scal + slot);
}

// Batches independent reductions into one pair of launches.
struct Reds {
  MultiRed m{};
  Reds(ahlp_problem_t p) {
    m.nred = 0;
    m.partial = p->ws.red_part;
    m.out = p->ws.scal;
  }
  Reds& add(int op, long long n, const double* a, const double* b, int slot,
            const double* c = nullptr, const double* d = nullptr, double s1 = 0, double s2 = 0) {
    RedSpec& r = m.r[m.nred++];
    r.op = op; r.slot = slot; r.n = n; r.a = a; r.b = b; r.c = c; r.d = d; r.s1 = s1; r.s2 = s2;
    return *this;
  }
  void launch(hipStream_t st) { launch_mreduce(st, m); }
};

// Refinement check of d = (dx, dy, dz) against r = (rx, ry, rz) on the
// unregularized Newton system (p->ws.g holds A'dy):  ex = rx - g - dz,
// ey = ry - A dx, ez = rz - Z dx - X dz.  With w2 the same row pass also
// forms aw2 = A (D dx dz / x) (the corrector's right-hand-side term).
void check_pass(ahlp_problem_t p, const double* rx, const double* ry, const double* rz,
                const double* dx, const double* dz, bool w2, hipStream_t st,
                const BndArgs* bnd = nullptr) {
  p->timer.begin(AHLP_ST_RESID);
  BndArgs b{};
  if (bnd) b = *bnd;
  b.q = p->qcur;
  launch_check_prep(st, p->blk, p->N, p->n0, p->x0off, p->d0off, rx, rz, p->ws.g, dx, dz, p->xs,
                    p->zs, p->Dp, p->ws.ex, p->ws.ez, p->ws.xp, w2 ? p->w2p : nullptr, b);
  RowsArgs ra{};
  ra.nv = 1;
  ra.v[0] = p->ws.xp; ra.base[0] = ry; ra.alpha[0] = -1.0; ra.out[0] = p->ws.ey; ra.with_C[0] = 1;
  if (w2) {
    ra.nv = 2;
    ra.v[1] = p->w2p; ra.alpha[1] = 1.0; ra.out[1] = p->aw2; ra.padded[1] = 1;
  }
  rows_pass(p, ra, st);
  link_global_rows(p, p->ws.xp, p->ws.xp + p->d0off, ry + p->mblk, -1.0, p->ws.ey + p->mblk, st);
  p->timer.end();
}

// max-abs reductions of the check (and of r on the first check)
void add_check_reds(ahlp_problem_t p, Reds& R, const double* rx, const double* ry,
                    const double* rz, const double* dx, const double* dy, const double* dz,
                    bool first) {
  R.add(RED_MAXABS, p->n_tot, p->ws.ex, nullptr, S_EN).add(RED_MAXABS, p->m_tot, p->ws.ey, nullptr, S_EN + 1)
      .add(RED_MAXABS, p->n_tot, p->ws.ez, nullptr, S_EN + 2).add(RED_MAXABS, p->n_tot, dx, nullptr, S_DN)
      .add(RED_MAXABS, p->m_tot, dy, nullptr, S_DN + 1).add(RED_MAXABS, p->n_tot, dz, nullptr, S_DN + 2);
  if (first)
    R.add(RED_MAXABS, p->n_tot, rx, nullptr, S_RN).add(RED_MAXABS, p->m_tot, ry, nullptr, S_RN + 1)
        .add(RED_MAXABS, p->n_tot, rz, nullptr, S_RN + 2);
}
double check_rn(ahlp_problem_t p) {
  const double* h = p->h_scal;
  return std::max(h[S_RN], std::max(h[S_RN + 1], h[S_RN + 2]));
}
// backward error |r - K d| / (|K| |d| + |r|) from the last check in h_scal
double check_bkerr(ahlp_problem_t p, double knorm, double rn) {
  const double* h = p->h_scal;
  const double en = std::max(h[S_EN], std::max(h[S_EN + 1], h[S_EN + 2]));
  const double dn = std::max(h[S_DN], std::max(h[S_DN + 1], h[S_DN + 2]));
  const double den = knorm * dn + rn;
  return den > 0 ? en / den : 0.0;
}

double check_en(ahlp_problem_t p) {
  const double* h = p->h_scal;
  return std::max(h[S_EN], std::max(h[S_EN + 1], h[S_EN + 2]));
}

// Iterative refinement from a checked d (its residual in ex, ey, ez):
// d += solve(e), g += A'c_y, re-check; until the backward error is at most
// tol (or the residual at most abs_tol, if abs_tol > 0) or max_refine
// corrections were applied.  With stagnate, a correction that reduces the
// backward error by less than 10x ends the loop.
ahlp_status_t refine(ahlp_problem_t p, const double* rx, const double* ry, const double* rz,
                     double* dx, double* dy, double* dz, int max_refine, double tol,
                     double knorm, double rn, bool w2, double* be, int* steps, hipStream_t st,
                     double abs_tol = 0.0, bool stagnate = false, const BndArgs* bnd = nullptr) {
  while (*be > tol && !(abs_tol > 0.0 && check_en(p) <= abs_tol) && *steps < max_refine) {
    const double be_prev = *be;
    CHK(solve_once(p, p->ws.ex, p->ws.ey, p->ws.ez, p->ws.cx, p->ws.cy, p->ws.cz, st, nullptr, p->ws.gc));
    launch_axpy(st, p->n_tot, 1.0, p->ws.cx, dx);
    launch_axpy(st, p->m_tot, 1.0, p->ws.cy, dy);
    launch_axpy(st, p->n_tot, 1.0, p->ws.cz, dz);
    launch_axpy(st, p->n_tot, 1.0, p->ws.gc, p->ws.g);
    check_pass(p, rx, ry, rz, dx, dz, w2, st, bnd);
    Reds R(p);
    add_check_reds(p, R, rx, ry, rz, dx, dy, dz, false);
    R.launch(st);
    CHK(read_scal(p, NSCAL, st));
    *be = check_bkerr(p, knorm, rn);
    ++*steps;
    if (stagnate && !(*be <= 0.1 * be_prev)) break;
  }
  return AHLP_OK;
}

// Refined solve.  d = (dx, dy, dz) receives the result.  knorm: |K|_inf.
ahlp_status_t solve_refined(ahlp_problem_t p, const double* rx, const double* ry,
                            const double* rz, double* dx, double* dy, double* dz, int max_refine,
                            double refine_tol, double knorm, double* bkerr, int* steps_out,
                            hipStream_t st) {
  CHK(solve_once(p, rx, ry, rz, dx, dy, dz, st));
  if (max_refine <= 0) {
    if (bkerr) *bkerr = -1.0;
    if (steps_out) *steps_out = 0;
    return AHLP_OK;
  }
  check_pass(p, rx, ry, rz, dx, dz, false, st);
  Reds R(p);
  add_check_reds(p, R, rx, ry, rz, dx, dy, dz, true);
  R.launch(st);
  CHK(read_scal(p, NSCAL, st));
  const double rn = check_rn(p);
  double be = check_bkerr(p, knorm, rn);
  int steps = 0;
  CHK(refine(p, rx, ry, rz, dx, dy, dz, max_refine, refine_tol, knorm, rn, false, &be, &steps, st));
  if (bkerr) *bkerr = be;
  if (steps_out) *steps_out = steps;
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

ahlp_status_t kkt_norm(ahlp_problem_t p, hipStream_t st, double* out) {
  red(p, RED_MAXSUM, p->n_tot, p->xs, p->zs, 9, st);
  if (p->qcur) red(p, RED_MAXABS, p->n_tot, p->qcur, nullptr, 8, st);
  HIPCHK(hipMemcpyAsync(p->h_scal + 8, p->ws.scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // |K|_inf: the (x) rows' |A| column sums + 1 (+ max q), the (y) rows, max(x + z)
  const double qmax = p->qcur ? p->h_scal[8] : 0.0;
  *out = std::max(p->colabs1_max + qmax, std::max(p->rowabs_max, p->h_scal[9]));
  return AHLP_OK;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

const char* ahlp_last_error(void) { return g_err.c_str(); }

void ahlp_ipm_default_opts(ahlp_ipm_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-8;
  o->max_iter = 100;
  o->eta = 0.99;
  o->rho = 1e-8;
  o->delta = 1e-6;
  o->max_refine = 5;
  o->refine_tol = 1e-10;
  o->precision = AHLP_FP64;
  o->mu_switch = 1e-6;
  o->start = 0;
  o->verbose = 0;
  o->timing = 0;
  o->fp32_accept = 0.1;
}

ahlp_status_t ahlp_problem_destroy(ahlp_problem_t p) {
  if (!p) return AHLP_OK;
  delete p;
  return AHLP_OK;
}

ahlp_status_t ahlp_problem_create(const ahlp_problem_desc_t* d, hipStream_t st,
                                  ahlp_problem_t* out) {
  g_err.clear();
  if (!d || !out) return fail(AHLP_EINVAL, "null argument");
  *out = nullptr;
  const int N = d->N, n0 = d->n0, ng = d->ng;
  if (N < 1) return fail(AHLP_EINVAL, "N must be >= 1 (got %d)", N);
  if (n0 < 0 || ng < 0 || ng + n0 > N0MAX)
    return fail(AHLP_EINVAL, "need n0 >= 0, ng >= 0 and ng + n0 <= %d (got n0=%d ng=%d)", N0MAX, n0, ng);
  if (ng > 0 && !d->Wg) return fail(AHLP_EINVAL, "ng > 0 needs Wg");
  const int nbw = ng + n0;   // width of the Schur border
  if (!d->m || !d->n || !d->A || !d->b || !d->c) return fail(AHLP_EINVAL, "missing m, n, A, b or c");
  if (N > 1 && (!d->l || !d->FR || !d->FL)) return fail(AHLP_EINVAL, "missing l, FR or FL");
  if (n0 > 0 && !d->C) return fail(AHLP_EINVAL, "n0 > 0 needs C");
  auto up = std::make_unique<ahlp_problem_s>();
  ahlp_problem_t p = up.get();
  HIPCHK(hipGetDevice(&p->device));
  p->N = N; p->n0 = n0; p->n0p = (int)r16(n0); p->P = N - 1;
  p->ng = ng; p->nb = nbw;
  p->m.assign(d->m, d->m + N);
  p->n.assign(d->n, d->n + N);
  if (N > 1) p->l.assign(d->l, d->l + N - 1);
  for (int i = 0; i < N; ++i)
    if (p->m[i] < 1 || p->n[i] < p->m[i])
      return fail(AHLP_EINVAL, "block %d: need 1 <= m <= n (m=%d n=%d)", i, p->m[i], p->n[i]);
  for (int j = 0; j < N - 1; ++j)
    if (p->l[j] < 0 || p->l[j] > LMAX || p->l[j] > std::min(p->n[j], p->n[j + 1]))
      return fail(AHLP_EINVAL, "pair %d: need 0 <= l <= min(n_j, n_j+1, %d) (l=%d)", j, LMAX, p->l[j]);
  p->lmax = 0;
  for (int v : p->l) p->lmax = std::max(p->lmax, v);
  int dev_lds = 0;
  HIPCHK(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  HIPCHK(hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, p->device));
  // the static workspace's address on this device (kept per device, resolved once)
  HIPCHK(scratch_setup(p->device));
  const size_t chain_sh = chain_factor_smem(std::max(p->lmax, 1), nbw);
  if (chain_sh > (size_t)dev_lds)
    return fail(AHLP_EINVAL,
                "link pairs (max %d) with a border of %d (global rows and linking variables) exceed "
                "the %d bytes of LDS", p->lmax, nbw, dev_lds);

  // ---- geometry
  long long xo = 0, yo = 0, dpo = 0, ao = 0, co = 0, lbo = 0, lio = 0, pqo = 0, vo = 0, qo = 0;
  p->loff.assign(std::max(N, 1), 0);
  for (int j = 0; j < N - 1; ++j) p->loff[j + 1] = p->loff[j] + p->l[j];
  p->nl = N > 1 ? p->loff[N - 1] : 0;
  const int kt0 = (nbw + 15) / 16, kc0 = (n0 + 15) / 16;
  p->hb.resize(N);
  int csr_off = 0, csc_off = 0;
  for (int i = 0; i < N; ++i) {
    BlockInfo& b = p->hb[i];
    b.m = p->m[i]; b.n = p->n[i];
    b.mt = (b.m + 15) / 16; b.nt = (b.n + 15) / 16;
    b.lL = i >= 1 ? p->l[i - 1] : 0;
    b.lR = i <= N - 2 ? p->l[i] : 0;
    b.ktL = (b.lL + 15) / 16; b.ktR = (b.lR + 15) / 16; b.kt0 = kt0;
    b.ng = ng; b.kc0 = kc0;
    b.kt = b.ktL + b.ktR + b.kt0;
    b.rt = b.mt + b.kt;
    b.pairL = i >= 1 ? i - 1 : -1;
    b.pairR = i <= N - 2 ? i : -1;
    b.csr_off = csr_off; csr_off += 16 * b.kt + 1;
    b.csc_off = csc_off; csc_off += b.n + 1;
    b.xoff = xo; xo += b.n;
    b.yoff = yo; yo += b.m;
    b.dpoff = dpo; dpo += 16LL * b.nt;
    b.aoff = ao; ao += 256LL * b.mt * b.nt;
    b.coff = co; co += 256LL * b.mt * b.kc0;
    b.lboff = lbo; lbo += 256LL * lb_tiles(b.mt, b.rt);
    b.linvoff = lio; lio += 256LL * b.mt;
    b.pqoff = pqo; pqo += 256LL * b.kt * b.kt;
    b.loffL = i >= 1 ? p->loff[i - 1] : -1;
    b.loffR = i <= N - 2 ? p->loff[i] : -1;
    b.voff = vo; vo += 16LL * b.mt;
    b.qoff = qo; qo += 16LL * b.kt;
    p->max_rt = std::max(p->max_rt, b.rt);
    p->max_kt = std::max(p->max_kt, b.kt);
  }
  // the column-at-a-time block factor keeps a bordered block's whole tile
  // column in LDS: (rt + 1) padded 16 x 17 tiles
  {
    const size_t col_sh = (size_t)(p->max_rt + 1) * 16 * 17 * sizeof(double);
    if (col_sh > (size_t)dev_lds)
      return fail(AHLP_EINVAL,
                  "a block with %d bordered tile rows (m_i + l_{i-1} + l_i + ng + n0 up to %d) needs %zu "
                  "bytes of LDS for its factorization; this device has %d (at most %d tile rows)",
                  p->max_rt, 16 * p->max_rt, col_sh, dev_lds, dev_lds / (16 * 17 * 8) - 1);
  }
  p->x0off = xo; p->n_tot = xo + n0;
  p->mblk = yo; p->nle = p->nl + ng; p->m_tot = yo + p->nle;
  p->d0off = dpo; p->dp_total = dpo + p->n0p;
  p->a_total = ao; p->c_total = co; p->lb_total = lbo; p->linv_total = lio; p->pq_total = pqo;
  p->vp_total = vo; p->q_total = qo;

  // ---- host packing: A and C into tile-major, link rows into CSR/CSC
  std::vector<double> hA((size_t)ao, 0.0), hC((size_t)std::max(co, 1LL), 0.0);
  std::vector<double> rowabs((size_t)p->m_tot, 0.0), colabs((size_t)p->n_tot, 0.0);
  {
    long long aoffs = 0, coffs = 0;
    for (int i = 0; i < N; ++i) {
      const BlockInfo& b = p->hb[i];
      const double* Ai = d->A + aoffs;
      for (int r = 0; r < b.m; ++r)
        for (int c = 0; c < b.n; ++c) {
          const double v = Ai[(long long)r * b.n + c];
          if (!std::isfinite(v)) return fail(AHLP_ENUMERIC, "non-finite A in block %d", i);
          hA[b.aoff + ((long long)(r / 16) * b.nt + c / 16) * 256 + (c % 16) * 16 + r % 16] = v;
          rowabs[b.yoff + r] += std::fabs(v);
          colabs[b.xoff + c] += std::fabs(v);
        }
      aoffs += (long long)b.m * b.n;
      if (n0 > 0) {
        const double* Ci = d->C + coffs;
        for (int r = 0; r < b.m; ++r)
          for (int c = 0; c < n0; ++c) {
            const double v = Ci[(long long)r * n0 + c];
            if (!std::isfinite(v)) return fail(AHLP_ENUMERIC, "non-finite C in block %d", i);
            hC[b.coff + ((long long)(r / 16) * kc0 + c / 16) * 256 + (c % 16) * 16 + r % 16] = v;
            rowabs[b.yoff + r] += std::fabs(v);
            colabs[p->x0off + c] += std::fabs(v);
          }
        coffs += (long long)b.m * n0;
      }
    }
  }
  // CSR of each block's link sections (rows q in [0, 16 kt), padded rows
  // empty): its part of the left and right pairs' link rows and of the global
  // rows (the border section's first ng rows)
  std::vector<int> hptr((size_t)csr_off, 0), hcol;
  std::vector<double> hval;
  std::vector<std::vector<std::pair<long long, double>>> colents((size_t)p->x0off);
  {
    long long froff = 0, floff = 0, wgoff = 0;
    std::vector<long long> fr_start(N > 1 ? N - 1 : 1, 0), fl_start(N > 1 ? N - 1 : 1, 0);
    for (int j = 0; j < N - 1; ++j) {
      fr_start[j] = froff; froff += (long long)p->l[j] * p->n[j];
      fl_start[j] = floff; floff += (long long)p->l[j] * p->n[j + 1];
    }
    for (int i = 0; i < N; ++i) {
      const BlockInfo& b = p->hb[i];
      for (int q = 0; q < 16 * b.kt; ++q) {
        hptr[b.csr_off + q] = (int)hcol.size();
        int qi;
        bool real;
        const int sec = link_section(b, q, &qi, nbw, &real);
        if (!real || !link_is_row(b, sec, qi)) continue;
        const double* row;
        long long grow;   // row inside the dual rows after the blocks (y_L, then y_G)
        if (sec == 2) {
          row = d->Wg + wgoff + (long long)qi * b.n;
          grow = p->nl + qi;
        } else {
          const int pair = sec == 0 ? i - 1 : i;
          row = sec == 0 ? d->FL + fl_start[pair] + (long long)qi * b.n
                         : d->FR + fr_start[pair] + (long long)qi * b.n;
          grow = p->loff[pair] + qi;
        }
        for (int c = 0; c < b.n; ++c) {
          const double v = row[c];
          if (v == 0.0) continue;
          if (!std::isfinite(v)) return fail(AHLP_ENUMERIC, "non-finite link coefficient");
          hcol.push_back(c);
          hval.push_back(v);
          colents[b.xoff + c].push_back({grow, v});
          rowabs[p->mblk + grow] += std::fabs(v);
          colabs[b.xoff + c] += std::fabs(v);
        }
      }
      hptr[b.csr_off + 16 * b.kt] = (int)hcol.size();
      wgoff += (long long)ng * b.n;
    }
  }
  // the global rows over the padded x, for the row passes
  std::vector<int> hgptr((size_t)ng + 1, 0), hgidx;
  std::vector<double> hgval;
  if (ng > 0) {
    if (dpo > (long long)INT32_MAX) return fail(AHLP_EINVAL, "padded x too long for the global rows' index");
    for (int k = 0; k < ng; ++k) {
      long long wgoff = 0;
      for (int i = 0; i < N; ++i) {
        const BlockInfo& b = p->hb[i];
        const double* row = d->Wg + wgoff + (long long)k * b.n;
        for (int c = 0; c < b.n; ++c)
          if (row[c] != 0.0) {
            hgidx.push_back((int)(b.dpoff + c));
            hgval.push_back(row[c]);
          }
        wgoff += (long long)ng * b.n;
      }
      hgptr[k + 1] = (int)hgidx.size();
    }
  }
  std::vector<int> hcptr((size_t)csc_off, 0), hcrow;
  std::vector<double> hcval;
  for (int i = 0; i < N; ++i) {
    const BlockInfo& b = p->hb[i];
    for (int c = 0; c < b.n; ++c) {
      hcptr[b.csc_off + c] = (int)hcrow.size();
      for (auto& e : colents[b.xoff + c]) {
        hcrow.push_back((int)e.first);
        hcval.push_back(e.second);
      }
    }
    hcptr[b.csc_off + b.n] = (int)hcrow.size();
  }
  // the x_0 coupling of the dual rows after the blocks: F0, then Wg0
  std::vector<double> hF0;
  p->f0first = p->nl;
  if (d->F0 && n0 > 0)
    for (long long r = 0; r < p->nl * n0; ++r)
      if (d->F0[r] != 0.0) {
        p->f0first = 0;
        break;
      }
  if (n0 > 0 && ((d->F0 && p->nl > 0) || (ng > 0 && d->Wg0))) {
    hF0.assign((size_t)(p->nle * n0), 0.0);
    if (d->F0)
      for (long long r = 0; r < p->nl; ++r)
        for (int c = 0; c < n0; ++c) hF0[r * n0 + c] = d->F0[r * n0 + c];
    if (ng > 0 && d->Wg0)
      for (long long r = 0; r < ng; ++r)
        for (int c = 0; c < n0; ++c) hF0[(p->nl + r) * n0 + c] = d->Wg0[r * n0 + c];
    for (long long r = 0; r < p->nle; ++r)
      for (int c = 0; c < n0; ++c) {
        const double v = hF0[r * n0 + c];
        if (!std::isfinite(v)) return fail(AHLP_ENUMERIC, r < p->nl ? "non-finite F0" : "non-finite Wg0");
        rowabs[p->mblk + r] += std::fabs(v);
        colabs[p->x0off + c] += std::fabs(v);
      }
  }
  for (long long i = 0; i < p->m_tot; ++i) {
    if (!std::isfinite(d->b[i])) return fail(AHLP_ENUMERIC, "non-finite b");
    p->b_inf = std::max(p->b_inf, std::fabs(d->b[i]));
  }
  for (long long i = 0; i < p->n_tot; ++i) {
    if (!std::isfinite(d->c[i])) return fail(AHLP_ENUMERIC, "non-finite c");
    p->c_inf = std::max(p->c_inf, std::fabs(d->c[i]));
  }
  std::vector<double> hub, hufin;
  if (d->ub) {
    for (long long i = 0; i < p->n_tot; ++i) {
      const double u = d->ub[i];
      if (std::isnan(u)) return fail(AHLP_ENUMERIC, "NaN upper bound");
      if (std::isfinite(u)) {
        if (!(u > 0.0)) return fail(AHLP_EINVAL, "upper bound %lld must be positive (got %g)", i, u);
        ++p->nU;
        p->ub_inf = std::max(p->ub_inf, u);
      } else if (u < 0.0) {
        return fail(AHLP_EINVAL, "upper bound %lld is -inf", i);
      }
    }
    if (p->nU > 0) {
      hub.assign(d->ub, d->ub + p->n_tot);
      hufin.resize((size_t)p->n_tot);
      for (long long i = 0; i < p->n_tot; ++i) hufin[i] = std::isfinite(hub[i]) ? hub[i] : 0.0;
    }
  }
  p->rowabs_max = 0.0;
  for (double v : rowabs) p->rowabs_max = std::max(p->rowabs_max, v);
  p->colabs1_max = 1.0;
  for (double v : colabs) p->colabs1_max = std::max(p->colabs1_max, v + 1.0);

  // ---- work lists
  // Uneven blocks: SYRK work goes largest block first, dealt round-robin into
  // eight chunks (the SYRK kernel gives each XCD a contiguous stretch of the
  // list, so every XCD gets a similar mix); the block factor runs two buckets
  // (panel kernel where the bordered block fits, column kernel otherwise),
  // each largest first.
  std::vector<int> bysize(N);
  for (int i = 0; i < N; ++i) bysize[i] = i;
  std::stable_sort(bysize.begin(), bysize.end(), [&](int a, int c) {
    const BlockInfo &x = p->hb[a], &y = p->hb[c];
    if (x.rt != y.rt) return x.rt > y.rt;
    if (x.mt != y.mt) return x.mt > y.mt;
    return x.nt > y.nt;
  });
  std::vector<int> syrk_order;
  for (int ch = 0; ch < 8; ++ch)
    for (int k = ch; k < N; k += 8) syrk_order.push_back(bysize[k]);
  p->bf_kernel.assign(p->max_rt + 1, -1);
  std::vector<int4> hsyrk;
  std::vector<int2> hlink, hrow, hcolt, hc0;
  p->syrk_off.assign(N, 0); p->syrk_cnt.assign(N, 0);
  p->link_off.assign(N, 0); p->link_cnt.assign(N, 0);
  for (int i : syrk_order) {
    const BlockInfo& b = p->hb[i];
    const int MT = (b.mt + 3) / 4;
    p->syrk_off[i] = (int)hsyrk.size();
    for (int r = 0; r < MT; ++r)
      for (int c = 0; c <= r; ++c) hsyrk.push_back(int4{i, r, c, 0});
    p->syrk_cnt[i] = (int)hsyrk.size() - p->syrk_off[i];
  }
  for (int i = 0; i < N; ++i) {
    const BlockInfo& b = p->hb[i];
    p->link_off[i] = (int)hlink.size();
    p->link_cnt[i] = b.kt;
    for (int r = 0; r < b.kt; ++r) hlink.push_back(int2{i, r});
    for (int r = 0; r < b.mt; ++r) hrow.push_back(int2{i, r});
    for (int c = 0; c < b.nt; ++c) hcolt.push_back(int2{i, c});
    for (int q = 0; q < b.kc0; ++q) hc0.push_back(int2{i, q});
  }
  p->nsyrk = (int)hsyrk.size(); p->nlink = (int)hlink.size();
  p->h_syrk = hsyrk;
  p->h_link = hlink;
  p->nrt = (int)hrow.size(); p->nct = (int)hcolt.size(); p->nc0 = (int)hc0.size();

  // ---- Schur complement geometry and segments
  const int P = p->P;
  p->tdoff.assign(std::max(P, 1), 0);
  p->tooff.assign(std::max(P, 1), 0);
  p->eoff.assign(std::max(P, 1), 0);
  p->zoff.assign(std::max(P, 1), 0);
  long long td = 0, to = 0, zo = 0;
  for (int j = 0; j < P; ++j) {
    p->tdoff[j] = td; td += (long long)p->l[j] * p->l[j];
    p->tooff[j] = to; if (j + 1 < P) to += (long long)p->l[j + 1] * p->l[j];
    p->eoff[j] = p->loff[j] * nbw;
  }
  if (P > 0) {
    int Ls = P <= 8 ? P : std::max(2, (int)std::lround(std::sqrt((double)P)));
    Ls = std::min(Ls, 24);
    int start = 0;
    while (start < P) {
      const int a = start;
      int bnd = std::min(start + Ls, P);
      if (bnd + 1 < P) {
        p->seg.push_back(int2{a, bnd});
        start = bnd + 1;
      } else {
        p->seg.push_back(int2{a, P});
        start = P;
      }
    }
  }
  p->G = (int)p->seg.size();
  for (int g = 0; g < p->G; ++g) {
    const int a = p->seg[g].x, b = p->seg[g].y;
    const int lsL = g > 0 ? p->l[a - 1] : 0;
    for (int k = a; k < b; ++k) { p->zoff[k] = zo; zo += (long long)lsL * p->l[k]; }
  }
  p->suboff.assign(std::max(p->G, 1), 0);
  long long so = 0;
  for (int s = 1; s < p->G - 1; ++s) {
    p->suboff[s] = so;
    so += (long long)p->l[p->seg[s].y] * p->l[p->seg[s - 1].y];
  }

  // ---- device allocations and uploads
  DevMem& M = p->mem;
  CHK(M.alloc(&p->blk, N));
  CHK(M.alloc(&p->A, ao));
  CHK(M.alloc(&p->C, std::max(co, 1LL)));
  CHK(M.alloc(&p->lptr, csr_off));
  CHK(M.alloc(&p->lcol, std::max<long long>(hcol.size(), 1)));
  CHK(M.alloc(&p->lval, std::max<long long>(hval.size(), 1)));
  CHK(M.alloc(&p->cptr, csc_off));
  CHK(M.alloc(&p->gptr, ng + 1));
  CHK(M.alloc(&p->gidx, std::max<long long>(hgidx.size(), 1)));
  CHK(M.alloc(&p->gval, std::max<long long>(hgval.size(), 1)));
  CHK(M.alloc(&p->crow, std::max<long long>(hcrow.size(), 1)));
  CHK(M.alloc(&p->cval, std::max<long long>(hcval.size(), 1)));
  if (!hF0.empty()) CHK(M.alloc(&p->F0, p->nle * n0));
  CHK(M.alloc(&p->b, p->m_tot));
  CHK(M.alloc(&p->c, p->n_tot));
  CHK(M.alloc(&p->syrk_items, p->nsyrk));
  CHK(M.alloc(&p->col_syrk_items, p->nsyrk));
  CHK(M.alloc(&p->col_link_items, std::max(p->nlink, 1)));
  CHK(M.alloc(&p->fused_queue, 1));
  CHK(M.alloc(&p->bf_order, N));
  CHK(M.alloc(&p->ident, N));
  CHK(M.alloc(&p->link_items, std::max(p->nlink, 1)));
  CHK(M.alloc(&p->rowtiles, p->nrt));
  CHK(M.alloc(&p->coltiles, p->nct));
  CHK(M.alloc(&p->c0tiles, std::max(p->nc0, 1)));
  CHK(M.alloc(&p->d_l, std::max(P, 1)));
  CHK(M.alloc(&p->d_loff, std::max(N, 1)));
  CHK(M.alloc(&p->d_tdoff, std::max(P, 1)));
  CHK(M.alloc(&p->d_tooff, std::max(P, 1)));
  CHK(M.alloc(&p->d_eoff, std::max(P, 1)));
  CHK(M.alloc(&p->d_zoff, std::max(P, 1)));
  CHK(M.alloc(&p->d_suboff, std::max(p->G, 1)));
  CHK(M.alloc(&p->d_seg, std::max(p->G, 1)));

  CHK(M.alloc(&p->Dp, p->dp_total));
  CHK(M.alloc(&p->xs, p->n_tot));
  CHK(M.alloc(&p->zs, p->n_tot));
  CHK(M.alloc(&p->LB, p->lb_total));
  CHK(M.alloc(&p->LINV, p->linv_total));
  CHK(M.alloc(&p->PQ, p->pq_total));
  CHK(M.alloc(&p->Td, std::max(td, 1LL)));
  CHK(M.alloc(&p->To, std::max(to, 1LL)));
  CHK(M.alloc(&p->E, std::max(p->nl * nbw, 1LL)));
  CHK(M.alloc(&p->S00, std::max(nbw * nbw, 1)));
  CHK(M.alloc(&p->thrT, std::max(P, 1)));
  CHK(M.alloc(&p->CL, std::max(td, 1LL)));
  CHK(M.alloc(&p->CLi, std::max(td, 1LL)));
  CHK(M.alloc(&p->CYn, std::max(to, 1LL)));
  CHK(M.alloc(&p->CZ, std::max(zo, 1LL)));
  CHK(M.alloc(&p->CG, std::max(p->nl * nbw, 1LL)));
  CHK(M.alloc(&p->CSub, std::max(so, 1LL)));
  CHK(M.alloc(&p->Lb, std::max(nbw * nbw, 1)));
  CHK(M.alloc(&p->Lbi, std::max(nbw * nbw, 1)));
  CHK(M.alloc(&p->S00w, std::max(nbw * nbw, 1)));
  p->tp = bcr_tiles(p->lmax, nbw);
  p->fast = p->tp > 0;
  for (int i = 0; i < N; ++i) {
    p->a_bytes += 8.0 * p->m[i] * p->n[i];
    p->c_bytes += 8.0 * p->m[i] * n0;
    p->xv_bytes += 8.0 * p->n[i];
    p->yv_bytes += 8.0 * p->m[i];
  }
  p->x0_bytes = 8.0 * n0;
  p->t0 = (nbw + 15) / 16;
  if (p->fast) {
    const long long Pt = std::max(P, 1);
    // chunks of at least 16 pairs, at most 64 chunks
    p->s00_chunk = std::max(16, (P + 63) / 64);
    p->s00_parts = P > 0 ? (P + p->s00_chunk - 1) / p->s00_chunk : 0;
    const long long T0 = std::max(p->t0, 1), tp = p->tp;
    for (double** v : {&p->BD, &p->BC, &p->FLi, &p->FXL, &p->FXR}) CHK(M.alloc(v, Pt * tp * tp * 256));
    CHK(M.alloc(&p->BEt, Pt * tp * T0 * 256));
    CHK(M.alloc(&p->FGt, Pt * tp * T0 * 256));
    CHK(M.alloc(&p->s00part, (long long)(p->s00_parts + 1) * std::max(p->t0 * p->t0, 1) * 256));
    CHK(M.alloc(&p->FLb, (long long)std::max(p->t0 * p->t0, 1) * 256));
    CHK(M.alloc(&p->FLbi, (long long)std::max(p->t0 * p->t0, 1) * 256));
    set_bcr_smem_limits();
    CHK(M.alloc(&p->segout, 1));
  } else {
    CHK(M.alloc(&p->segout, (long long)std::max(p->G, 1) * SEG_STRIDE));
  }

  {
    double* wsbuf = nullptr;
    CHK(M.alloc(&wsbuf, (long long)(solve_ws_layout(p, nullptr, nullptr) / sizeof(double))));
    solve_ws_layout(p, wsbuf, &p->ws);
  }
  p->info = reinterpret_cast<DevInfo*>(p->ws.scal + NSCAL - 1);
  for (double** v : {&p->ones, &p->zerosn, &p->rd, &p->rzv, &p->dxa, &p->dza, &p->dx, &p->dz})
    CHK(M.alloc(v, p->n_tot));
  for (double** v : {&p->rp, &p->dya, &p->dy}) CHK(M.alloc(v, p->m_tot));
  for (double** v : {&p->ta, &p->aw1, &p->aw2, &p->tc}) CHK(M.alloc(v, p->vp_total));
  for (double** v : {&p->w1p, &p->w2p}) CHK(M.alloc(v, p->dp_total));
  CHK(M.alloc(&p->aty, p->n_tot));
  CHK(M.alloc(&p->gdir, p->n_tot));
  CHK(M.alloc(&p->adj_rz, p->n_tot));
  CHK(M.alloc(&p->grad_g, p->n_tot));
  CHK(M.alloc(&p->grad_wz, p->n_tot));
  for (double** v : {&p->g_r, &p->g_dx, &p->g_dz}) CHK(M.alloc(v, p->n_tot));
  for (double** v : {&p->g_dy, &p->zerosm}) CHK(M.alloc(v, p->m_tot));
  if (p->nU > 0) {
    for (double** v : {&p->ub, &p->ufin, &p->bs, &p->bw, &p->bdsa, &p->bdwa, &p->bds, &p->bdw,
                       &p->bru, &p->bq, &p->bzw, &p->brdt, &p->brxc, &p->bsm, &p->bwm})
      CHK(M.alloc(v, p->n_tot));
    HIPCHK(hipMemcpyAsync(p->ub, hub.data(), sizeof(double) * p->n_tot, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->ufin, hufin.data(), sizeof(double) * p->n_tot, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipHostMalloc((void**)&p->h_scal, NSCAL * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&p->ev_gin, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_gout, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));

  HIPCHK(hipMemcpyAsync(p->blk, p->hb.data(), sizeof(BlockInfo) * N, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->A, hA.data(), sizeof(double) * ao, hipMemcpyHostToDevice, st));
  if (co > 0) HIPCHK(hipMemcpyAsync(p->C, hC.data(), sizeof(double) * co, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->lptr, hptr.data(), sizeof(int) * csr_off, hipMemcpyHostToDevice, st));
  if (!hcol.empty()) {
    HIPCHK(hipMemcpyAsync(p->lcol, hcol.data(), sizeof(int) * hcol.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->lval, hval.data(), sizeof(double) * hval.size(), hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(p->cptr, hcptr.data(), sizeof(int) * csc_off, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->gptr, hgptr.data(), sizeof(int) * (ng + 1), hipMemcpyHostToDevice, st));
  if (!hgidx.empty()) {
    HIPCHK(hipMemcpyAsync(p->gidx, hgidx.data(), sizeof(int) * hgidx.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->gval, hgval.data(), sizeof(double) * hgval.size(), hipMemcpyHostToDevice, st));
  }
  if (!hcrow.empty()) {
    HIPCHK(hipMemcpyAsync(p->crow, hcrow.data(), sizeof(int) * hcrow.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->cval, hcval.data(), sizeof(double) * hcval.size(), hipMemcpyHostToDevice, st));
  }
  if (p->F0) HIPCHK(hipMemcpyAsync(p->F0, hF0.data(), sizeof(double) * p->nle * n0, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->b, d->b, sizeof(double) * p->m_tot, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->c, d->c, sizeof(double) * p->n_tot, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->syrk_items, hsyrk.data(), sizeof(int4) * hsyrk.size(), hipMemcpyHostToDevice, st));
  {
    std::vector<int> id(N);
    for (int i = 0; i < N; ++i) id[i] = i;
    HIPCHK(hipMemcpyAsync(p->ident, id.data(), sizeof(int) * N, hipMemcpyHostToDevice, st));
  }
  if (!hlink.empty())
    HIPCHK(hipMemcpyAsync(p->link_items, hlink.data(), sizeof(int2) * hlink.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->rowtiles, hrow.data(), sizeof(int2) * hrow.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->coltiles, hcolt.data(), sizeof(int2) * hcolt.size(), hipMemcpyHostToDevice, st));
  if (!hc0.empty())
    HIPCHK(hipMemcpyAsync(p->c0tiles, hc0.data(), sizeof(int2) * hc0.size(), hipMemcpyHostToDevice, st));
  if (P > 0) {
    HIPCHK(hipMemcpyAsync(p->d_l, p->l.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_tdoff, p->tdoff.data(), sizeof(long long) * P, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_tooff, p->tooff.data(), sizeof(long long) * P, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_eoff, p->eoff.data(), sizeof(long long) * P, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_zoff, p->zoff.data(), sizeof(long long) * P, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(p->d_loff, p->loff.data(), sizeof(long long) * std::max(N, 1), hipMemcpyHostToDevice, st));
  if (p->G > 0) {
    HIPCHK(hipMemcpyAsync(p->d_seg, p->seg.data(), sizeof(int2) * p->G, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_suboff, p->suboff.data(), sizeof(long long) * p->G, hipMemcpyHostToDevice, st));
  }
  launch_fill(st, p->n_tot, 1.0, p->ones);
  launch_fill(st, p->m_tot, 0.0, p->zerosm);
  launch_fill(st, p->n_tot, 0.0, p->zerosn);
  static_assert(sizeof(DevInfo) <= sizeof(double), "DevInfo lives in one scalar slot");
  launch_fill(st, 1, 0.0, reinterpret_cast<double*>(p->info));   // a kernel, not a memset: capturable
  if (chain_sh > 64 * 1024) set_chain_smem_limits(chain_sh);
  HIPCHK(hipGetLastError());
  CHK(set_buckets(p, st));
  HIPCHK(hipStreamSynchronize(st));
  p->timer.st = st;
  *out = up.release();
  return AHLP_OK;
}

ahlp_status_t ahlp_kkt_factor(ahlp_problem_t p, const double* x, const double* z,
                              const ahlp_factor_opts_t* o, hipStream_t st) {
  g_err.clear();
  if (!p || !x || !z) return fail(AHLP_EINVAL, "null argument");
  const int prec = o ? o->precision : AHLP_FP64;
  const double rho = o ? o->rho : 0.0, delta = o ? o->delta : 0.0;
  if (!(rho >= 0.0) || !(delta >= 0.0)) return fail(AHLP_EINVAL, "rho and delta must be >= 0");
  if (prec != AHLP_FP64 && prec != AHLP_FP32_REFINE) return fail(AHLP_EINVAL, "unknown precision");
  p->timer.st = st;
  p->qcur = nullptr;
  return do_factor(p, x, z, prec, rho, delta, st);
}

ahlp_status_t ahlp_kkt_factor_bounded(ahlp_problem_t p, const double* x, const double* z,
                                      const double* q, const ahlp_factor_opts_t* o,
                                      hipStream_t st) {
  g_err.clear();
  if (!p || !x || !z || !q) return fail(AHLP_EINVAL, "null argument");
  const int prec = o ? o->precision : AHLP_FP64;
  const double rho = o ? o->rho : 0.0, delta = o ? o->delta : 0.0;
  if (!(rho >= 0.0) || !(delta >= 0.0)) return fail(AHLP_EINVAL, "rho and delta must be >= 0");
  if (prec != AHLP_FP64 && prec != AHLP_FP32_REFINE) return fail(AHLP_EINVAL, "unknown precision");
  if (!p->bqapi) CHK(p->mem.alloc(&p->bqapi, p->n_tot));
  p->timer.st = st;
  launch_copy(st, p->n_tot, q, p->bqapi);
  p->qcur = p->bqapi;
  return do_factor(p, x, z, prec, rho, delta, st);
}

ahlp_status_t ahlp_ipm_bound_duals(ahlp_problem_t p, double* s, double* w, hipStream_t st) {
  g_err.clear();
  if (!p) return fail(AHLP_EINVAL, "null handle");
  if (!p->ub) return fail(AHLP_ESTATE, "the problem has no upper bounds");
  if (s) launch_copy(st, p->n_tot, p->bs, s);
  if (w) launch_copy(st, p->n_tot, p->bw, w);
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

namespace {
// ahlp_kkt_solve on the handle's current workspace p->ws.
ahlp_status_t kkt_solve_impl(ahlp_problem_t p, const double* rx, const double* ry,
                             const double* rz, double* dx, double* dy, double* dz,
                             int32_t max_refine, double refine_tol, double* bkerr,
                             hipStream_t st) {
  if (!p || !rx || !ry || !rz || !dx || !dy || !dz) return fail(AHLP_EINVAL, "null argument");
  if (!p->factored) return fail(AHLP_ESTATE, "solve before factor");
  p->timer.st = st;
  if (max_refine > 0) {
    bool bad = false;
    CHK(check_info(p, st, &bad));
    if (bad) return fail(AHLP_ENUMERIC, "the factorization saw x <= 0, z <= 0 or non-finite values");
    double kn = 0;
    CHK(kkt_norm(p, st, &kn));
    return solve_refined(p, rx, ry, rz, dx, dy, dz, max_refine, refine_tol, kn, bkerr, nullptr, st);
  }
  return solve_once(p, rx, ry, rz, dx, dy, dz, st);
}
}  // namespace

ahlp_status_t ahlp_kkt_solve(ahlp_problem_t p, const double* rx, const double* ry,
                             const double* rz, double* dx, double* dy, double* dz,
                             int32_t max_refine, double refine_tol, double* bkerr,
                             hipStream_t st) {
  g_err.clear();
  return kkt_solve_impl(p, rx, ry, rz, dx, dy, dz, max_refine, refine_tol, bkerr, st);
}

ahlp_status_t ahlp_kkt_solve_noalloc(ahlp_problem_t p, const double* rx, const double* ry,
                                     const double* rz, double* dx, double* dy, double* dz,
                                     int32_t max_refine, double refine_tol, double* bkerr,
                                     hipStream_t st) {
  g_err.clear();
  if (!p) return fail(AHLP_EINVAL, "null argument");
  double* base = scratch_device_ptr(p->device);
  if (!base) return fail(AHLP_ESTATE, "the static workspace of device %d was not set up", p->device);
  const size_t need = solve_ws_layout(p, nullptr, nullptr);
  if (need > SCRATCH_BYTES)
    return fail(AHLP_EINVAL,
                "this problem's solve needs %zu bytes of workspace; the static workspace holds %zu "
                "(use ahlp_kkt_solve)", need, (size_t)SCRATCH_BYTES);
  SolveWs mine{};
  solve_ws_layout(p, base, &mine);
  // the array keeps the previous call's contents: start from zeros (a fill
  // kernel, no memset node if the caller captures the stream)
  launch_fill(st, (long long)(need / sizeof(double)), 0.0, base);
  HIPCHK(hipGetLastError());
  const SolveWs saved = p->ws;
  p->ws = mine;
  const ahlp_status_t s =
      kkt_solve_impl(p, rx, ry, rz, dx, dy, dz, max_refine, refine_tol, bkerr, st);
  p->ws = saved;
  return s;
}

ahlp_status_t ahlp_kkt_adjoint(ahlp_problem_t p, const double* gx, const double* gy,
                               const double* gz, double* wx, double* wy, double* wz,
                               int32_t max_refine, double refine_tol, double* bkerr,
                               hipStream_t st) {
  g_err.clear();
  if (!p || !gx || !gy || !gz || !wx || !wy || !wz) return fail(AHLP_EINVAL, "null argument");
  if (!p->factored) return fail(AHLP_ESTATE, "adjoint solve before factor");
  if (wx == gx || wy == gy || wz == gz) return fail(AHLP_EINVAL, "outputs must not alias inputs");
  // K' w = g  <=>  K (wx, wy, z wz) = (gx, gy, z gz)
  launch_adj_scale(st, p->n_tot, 0, p->zs, gz, p->adj_rz);
  HIPCHK(hipGetLastError());
  CHK(ahlp_kkt_solve(p, gx, gy, p->adj_rz, wx, wy, wz, max_refine, refine_tol, bkerr, st));
  launch_adj_scale(st, p->n_tot, 1, p->zs, wz, wz);
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

ahlp_status_t ahlp_lp_gradient(ahlp_problem_t p, const double* gx, double gf, double* grad_b,
                               double* grad_c, int32_t max_refine, double refine_tol,
                               double* bkerr, hipStream_t st) {
  g_err.clear();
  if (!p || !grad_b || !grad_c) return fail(AHLP_EINVAL, "null argument");
  if (!p->factored) return fail(AHLP_ESTATE, "gradient before factor");
  if (!std::isfinite(gf)) return fail(AHLP_EINVAL, "dL/df must be finite");
  if (gx == grad_c) return fail(AHLP_EINVAL, "outputs must not alias inputs");
  // g_x = dL/dx + (dL/df) c
  if (gx) launch_copy(st, p->n_tot, gx, p->grad_g);
  else launch_fill(st, p->n_tot, 0.0, p->grad_g);
  if (gf != 0.0) launch_axpy(st, p->n_tot, gf, p->c, p->grad_g);
  HIPCHK(hipGetLastError());
  CHK(ahlp_kkt_adjoint(p, p->grad_g, p->zerosm, p->zerosn, grad_c, grad_b, p->grad_wz, max_refine,
                       refine_tol, bkerr, st));
  // dL/dc = w_x + (dL/df) x at the factorization's x
  if (gf != 0.0) launch_axpy(st, p->n_tot, gf, p->xs, grad_c);
  HIPCHK(hipGetLastError());
  return AHLP_OK;
}

namespace {
std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}
}  // namespace

ahlp_status_t ahlp_autotune(ahlp_problem_t p, const char* cache_path, int32_t* measured,
                            hipStream_t st) {
  g_err.clear();
  if (!p) return fail(AHLP_EINVAL, "null argument");
  if (measured) *measured = 0;
  const std::string arch = arch_name(p->device);
  // rt values with a choice to make (at least two kernels can hold them)
  std::vector<int> todo;
  for (int rt = 1; rt <= p->max_rt; ++rt) {
    if (!block_factor_panel8_fits(rt)) continue;
    bool present = false;
    for (const auto& b : p->hb) present = present || b.rt == rt;
    if (present) todo.push_back(rt);
  }
  // cached entries: "<arch> <rt> <panel|column|panel8> <us panel> <us column> [<us panel8>]"
  // (a time of -1: the kernel cannot hold blocks of that rt)
  static const char* names[3] = {"panel", "column", "panel8"};
  std::vector<std::string> keep;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string a, k;
      int rt = 0;
      if (line.empty() || line[0] == '#' || !(ls >> a >> rt >> k)) continue;
      keep.push_back(line);
      if (a != arch || rt < 1 || rt > p->max_rt) continue;
      for (int q = 0; q < 3; ++q)
        if (k == names[q]) p->bf_kernel[rt] = q;
    }
  }
  std::vector<int> need;
  for (int rt : todo)
    if (p->bf_kernel[rt] < 0) need.push_back(rt);
  std::vector<std::string> fresh;
  if (!need.empty()) {
    // inputs of the block factor at x = z = 1: D, then M_i and B_i' rebuilt
    // by the SYRK and the link gather before every timed launch
    const int saved_mode = p->launch_mode;
    const double rho = 1e-8, delta = 1e-6;
    p->delta = delta;
    launch_fill(st, p->n_tot, 1.0, p->ones);
    CHK(prep_scaling(p, p->ones, p->ones, rho, st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::vector<int> hblk;
    for (int rt : need) {
      hblk.clear();
      for (int i = 0; i < p->N; ++i)
        if (p->hb[i].rt == rt) hblk.push_back(i);
      HIPCHK(hipMemcpyAsync(p->bf_order, hblk.data(), sizeof(int) * hblk.size(), hipMemcpyHostToDevice, st));
      double best[3] = {1e30, 1e30, 1e30};
      const bool can[3] = {block_factor_panel_fits(rt), true, block_factor_panel8_fits(rt)};
      for (int rep = 0; rep < 2; ++rep)
        for (int k = 0; k < 3; ++k) {
          if (!can[k]) continue;
          launch_link<double>(st, p->blk, p->link_items, p->nlink, p->nb, p->A, p->C, p->lptr,
                              p->lcol, p->lval, p->Dp, p->LB, p->PQ);
          launch_syrk<double>(st, p->blk, p->syrk_items, p->nsyrk, p->A, p->Dp, p->LB, delta);
          HIPCHK(hipEventRecord(e0, st));
          if (k == BFK_COLUMN)
            launch_block_factor_col<double>(st, p->blk, p->bf_order, (int)hblk.size(), rt, p->LB,
                                            p->LINV, p->PQ, p->info);
          else
            launch_block_factor_panel<double>(st, p->blk, p->bf_order, (int)hblk.size(), rt, p->LB,
                                              p->LINV, p->PQ, p->info, k == BFK_PANEL8 ? 8 : 4,
                                              p->max_kt);
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          best[k] = std::min(best[k], 1e3 * (double)ms);
        }
      // decided on the values the cache records (to the nanosecond), so a
      // table read back agrees with its own timings
      int pick = -1;
      for (int k = 0; k < 3; ++k) {
        if (!can[k]) continue;
        best[k] = std::round(best[k] * 1e3) / 1e3;
        if (pick < 0 || best[k] < best[pick]) pick = k;
      }
      p->bf_kernel[rt] = pick;
      char buf[192];
      std::snprintf(buf, sizeof buf, "%s %d %s %.3f %.3f %.3f", arch.c_str(), rt, names[pick],
                    can[0] ? best[0] : -1.0, best[1], can[2] ? best[2] : -1.0);
      fresh.push_back(buf);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->launch_mode = saved_mode;
    p->factored = false;   // the tuning runs overwrote the factors
    if (measured) *measured = (int32_t)need.size();
    if (cache_path) {
      std::ofstream out(cache_path);
      out << "# block-factor kernel per bordered tile-row count: arch rt kernel us_panel us_column "
             "us_panel8\n";
      for (const auto& l : keep) out << l << "\n";
      for (const auto& l : fresh) out << l << "\n";
      if (!out) return fail(AHLP_EINVAL, "cannot write the tuning cache %s", cache_path);
    }
  }
  // The choices per rt are measured one rt at a time; run together, buckets
  // interact (a small bucket of eight-wave workgroups holds whole CUs that the
  // large four-wave bucket beside it would use).  So the whole factorization
  // is timed with the tuned choices and with the default rule, and the
  // faster plan is kept.
  {
    const std::vector<int> tuned = p->bf_kernel;
    bool differs = false;
    for (int rt = 1; rt <= p->max_rt; ++rt) {
      const int k = tuned[rt];
      std::vector<int> dflt(p->max_rt + 1, -1);
      std::swap(p->bf_kernel, dflt);
      const int d = bf_choice(p, rt);
      std::swap(p->bf_kernel, dflt);
      bool present = false;
      for (const auto& b : p->hb) present = present || b.rt == rt;
      if (present && k >= 0 && k != d) differs = true;
    }
    if (differs) {
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      const int saved_mode = p->launch_mode;
      p->launch_mode = AHLP_LAUNCH_BATCHED;
      p->delta = 1e-6;
      launch_fill(st, p->n_tot, 1.0, p->ones);
      CHK(prep_scaling(p, p->ones, p->ones, 1e-8, st));
      double t_plan[2] = {1e30, 1e30};
      for (int rep = 0; rep < 3; ++rep)
        for (int q = 0; q < 2; ++q) {
          if (q == 0) p->bf_kernel = tuned;
          else p->bf_kernel.assign(p->max_rt + 1, -1);
          CHK(set_buckets(p, st));
          HIPCHK(hipEventRecord(e0, st));
          CHK(factor_blocks<double>(p, st, p->LB, p->LINV, p->A));
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) t_plan[q] = std::min(t_plan[q], (double)ms);   // rep 0 warms up
        }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      p->launch_mode = saved_mode;
      p->factored = false;
      if (t_plan[0] <= t_plan[1]) p->bf_kernel = tuned;
      else p->bf_kernel.assign(p->max_rt + 1, -1);
    }
  }
  CHK(set_buckets(p, st));   // (captured graphs hold the old buckets: they are captured again)
  return AHLP_OK;
}

ahlp_status_t ahlp_problem_set_launch(ahlp_problem_t p, int32_t mode) {
  g_err.clear();
  if (!p) return fail(AHLP_EINVAL, "null argument");
  if (mode != AHLP_LAUNCH_BATCHED && mode != AHLP_LAUNCH_PER_BLOCK && mode != AHLP_LAUNCH_FUSED)
    return fail(AHLP_EINVAL, "unknown launch mode %d", mode);
  if (mode != p->launch_mode) ++p->launch_gen;
  p->launch_mode = mode;
  return AHLP_OK;
}

ahlp_status_t ahlp_problem_set_bc(ahlp_problem_t p, const double* b, const double* c,
                                  hipStream_t st) {
  g_err.clear();
  if (!p || !b || !c) return fail(AHLP_EINVAL, "null argument");
  HIPCHK(hipMemcpyAsync(p->b, b, sizeof(double) * p->m_tot, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(p->c, c, sizeof(double) * p->n_tot, hipMemcpyDeviceToDevice, st));
  // max |b|, max |c| for the stopping test; the sums of squares catch NaN
  Reds(p).add(RED_MAXABS, p->m_tot, p->b, nullptr, 0).add(RED_MAXABS, p->n_tot, p->c, nullptr, 1)
      .add(RED_DOT, p->m_tot, p->b, p->b, 2).add(RED_DOT, p->n_tot, p->c, p->c, 3).launch(st);
  HIPCHK(hipGetLastError());
  CHK(read_scal(p, 4, st));
  const double* h = p->h_scal;
  if (!std::isfinite(h[2]) || !std::isfinite(h[3]))
    return fail(AHLP_ENUMERIC, "b or c has non-finite entries");
  p->b_inf = h[0];
  p->c_inf = h[1];
  return AHLP_OK;
}

ahlp_status_t ipm_solve_impl(ahlp_problem_t p, const ahlp_ipm_opts_t* o, double* x, double* y,
                             double* z, ahlp_ipm_result_t* res, hipStream_t st);

ahlp_status_t ahlp_ipm_solve(ahlp_problem_t p, const ahlp_ipm_opts_t* o, double* x, double* y,
                             double* z, ahlp_ipm_result_t* res, hipStream_t st) {
  g_err.clear();
  if (!p || !o || !x || !y || !z) return fail(AHLP_EINVAL, "null argument");
  if (o->graph && !o->timing) {
    // graph mode: run on the library's capturable stream, ordered after and
    // before the caller's stream by events
    HIPCHK(hipEventRecord(p->ev_gin, st));
    HIPCHK(hipStreamWaitEvent(p->gstream, p->ev_gin, 0));
    p->use_graph = true;
    const ahlp_status_t s = ipm_solve_impl(p, o, x, y, z, res, p->gstream);
    p->use_graph = false;
    HIPCHK(hipEventRecord(p->ev_gout, p->gstream));
    HIPCHK(hipStreamWaitEvent(st, p->ev_gout, 0));
    return s;
  }
  return ipm_solve_impl(p, o, x, y, z, res, st);
}

ahlp_status_t ipm_solve_impl(ahlp_problem_t p, const ahlp_ipm_opts_t* o, double* x, double* y,
                             double* z, ahlp_ipm_result_t* res, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  ahlp_ipm_result_t R;
  std::memset(&R, 0, sizeof R);
  p->timer.st = st;
  p->timer.on = o->timing != 0;
  // timing 2: the factorization stages a1-a5 only (fewer events in the stream)
  p->timer.mask = o->timing == 2 ? ((1u << AHLP_ST_PREP) | (1u << AHLP_ST_SYRK) |
                                    (1u << AHLP_ST_FACTOR) | (1u << AHLP_ST_SCHUR))
                                 : ~0u;
  p->timer.reset();
  p->rows_bytes = 0.0;
  p->hist.clear();
  R.start_bkerr[0] = R.start_bkerr[1] = -1.0;
  const long long n = p->n_tot, m = p->m_tot;
  const bool bnd = p->nU > 0;
  if (bnd && o->gondzio > 0)
    return fail(AHLP_EINVAL, "Gondzio correctors are not combined with upper bounds");
  p->qcur = nullptr;   // the start point's factorization has no bound term
  int total_piv = 0;
  double max_bk = 0.0;
  int refine_total = 0;
  auto account = [&](double be, int steps) {
    refine_total += steps;
    if (be > max_bk) max_bk = be;
  };
  auto factor_checked = [&](const double* xx, const double* zz, int prec, double rho,
                            double delta) -> ahlp_status_t {
    CHK(do_factor(p, xx, zz, prec, rho, delta, st));
    bool bad = false;
    CHK(check_info(p, st, &bad));
    p->timer.collect();
    total_piv += p->pivots_seen;
    if (bad) return fail(AHLP_ENUMERIC, "x or z left the positive orthant or became non-finite");
    return AHLP_OK;
  };

  // ---- starting point
  if (o->start == 0) {
    CHK(factor_checked(p->ones, p->ones, AHLP_FP64, 0.0, 0.0));
    double kn = 0;
    CHK(kkt_norm(p, st, &kn));
    double be;
    int steps;
    // x~ from rhs (0, b, 0), y~ from rhs (c, 0, 0)
    CHK(solve_refined(p, p->zerosn, p->b, p->zerosn, p->dxa, p->dya, p->dza, o->max_refine,
                      o->refine_tol, kn, &be, &steps, st));
    account(be, steps);
    R.start_bkerr[0] = be;
    HIPCHK(hipMemsetAsync(p->rp, 0, sizeof(double) * m, st));
    CHK(solve_refined(p, p->c, p->rp, p->zerosn, p->dx, p->dy, p->dz, o->max_refine,
                      o->refine_tol, kn, &be, &steps, st));
    account(be, steps);
    R.start_bkerr[1] = be;
    launch_copy(st, n, p->dxa, x);
    launch_copy(st, m, p->dy, y);
    apply_At(p, y, 1, p->c, p->zerosn, z, st);   // z~ = c - A'y~
    if (bnd) {
      // bounded variables: z = max(z~, 0), w = max(-z~, 0), s = u - x~; the
      // pairs (x, s) and (z, w) shifted and centred together
      launch_bnd_start(st, n, p->ub, x, z, p->bs, p->bw, p->bsm, p->bwm);
      Reds(p).add(RED_MIN, n, x, nullptr, 0).add(RED_MIN, n, p->bsm, nullptr, 1)
          .add(RED_MIN, n, z, nullptr, 2).add(RED_MIN, n, p->bwm, nullptr, 3).launch(st);
      CHK(read_scal(p, 4, st));
      const double mp = std::min(p->h_scal[0], p->h_scal[1]), md = std::min(p->h_scal[2], p->h_scal[3]);
      launch_bnd_shift(st, n, p->ub, std::max(-1.5 * mp, 0.0), std::max(-1.5 * md, 0.0), x, z, p->bs,
                       p->bw, p->bsm, p->bwm);
      Reds(p).add(RED_DOT, n, x, z, 0).add(RED_DOT, n, p->bs, p->bw, 1)
          .add(RED_DOT, n, x, p->ones, 2).add(RED_DOT, n, p->bs, p->ones, 3)
          .add(RED_DOT, n, z, p->ones, 4).add(RED_DOT, n, p->bw, p->ones, 5).launch(st);
      CHK(read_scal(p, 6, st));
      const double* hh = p->h_scal;
      const double xz = hh[0] + hh[1], sx = hh[2] + hh[3], sz = hh[4] + hh[5];
      launch_bnd_shift(st, n, p->ub, sz > 0 ? 0.5 * xz / sz : 0.0, sx > 0 ? 0.5 * xz / sx : 0.0, x, z,
                       p->bs, p->bw, p->bsm, p->bwm);
      Reds(p).add(RED_MIN, n, x, nullptr, 0).add(RED_MIN, n, z, nullptr, 1)
          .add(RED_MIN, n, p->bsm, nullptr, 2).add(RED_MIN, n, p->bwm, nullptr, 3).launch(st);
      CHK(read_scal(p, 4, st));
      if (hh[0] <= 0.0 || hh[1] <= 0.0 || hh[2] <= 0.0 || hh[3] <= 0.0)
        launch_bnd_shift(st, n, p->ub, 1.0, 1.0, x, z, p->bs, p->bw, p->bsm, p->bwm);
    }
    Reds(p).add(RED_MIN, n, x, nullptr, 0).add(RED_MIN, n, z, nullptr, 1).launch(st);
    CHK(read_scal(p, 2, st));
    if (!bnd) {
      const double sx = std::max(-1.5 * p->h_scal[0], 0.0), sz = std::max(-1.5 * p->h_scal[1], 0.0);
      launch_addscalar(st, n, sx, x);
      launch_addscalar(st, n, sz, z);
      Reds(p).add(RED_DOT, n, x, z, 0).add(RED_DOT, n, x, p->ones, 1).add(RED_DOT, n, z, p->ones, 2)
          .launch(st);
      CHK(read_scal(p, 3, st));
      const double xz = p->h_scal[0], sumx = p->h_scal[1], sumz = p->h_scal[2];
      launch_addscalar(st, n, sumz > 0 ? 0.5 * xz / sumz : 0.0, x);
      launch_addscalar(st, n, sumx > 0 ? 0.5 * xz / sumx : 0.0, z);
      Reds(p).add(RED_MIN, n, x, nullptr, 0).add(RED_MIN, n, z, nullptr, 1).launch(st);
      CHK(read_scal(p, 2, st));
      if (p->h_scal[0] <= 0.0 || p->h_scal[1] <= 0.0) {
        launch_addscalar(st, n, 1.0, x);
        launch_addscalar(st, n, 1.0, z);
      }
    }
  } else if (bnd) {
    return fail(AHLP_EINVAL, "a problem with upper bounds starts from its own start point (start = 0)");
  }

  // ---- main loop
  // One iteration: a column pass for r_d, one row pass that forms r_p = b - A x,
  // the predictor's t_a = r_p + A D rhx_a and A (D/x); the factorization; the
  // predictor solve and its check (whose row pass also forms A (D dxa dza / x));
  // the corrector's t_c = t_a - sigma mu A(D/x) + A(D dxa dza / x), which is
  // its rhs term r_p + A D rhx_c written out by linearity (rhx = rx - rz / x);
  // the corrector solve and check.  The host waits three times: after the
  // residuals, after the predictor's check with its step lengths and mu_aff,
  // and after the corrector's check with its step lengths.
  const double bn = 1.0 + p->b_inf, cn = 1.0 + p->c_inf;
  bool fp32_live = o->precision == AHLP_FP32_REFINE;
  int k = 0;
  ahlp_status_t status = AHLP_WMAXITER;
  double mu = 0, pobj = 0, dobj = 0, relgap = 0, pinf = 0, dinf = 0;
  const DevInfo* hinfo = reinterpret_cast<const DevInfo*>(p->h_scal + NSCAL - 1);
  const double* hs = p->h_scal;
  SegKey key{x, y, z, o->rho, o->delta, o->eta, p->launch_gen};
  // residuals of the current iterate (the start of every iteration).  A'y is
  // kept in p->aty: formed by a column pass at the start (full), then
  // advanced with each step, A'y+ = A'y + alpha_d A'dy, where A'dy is the
  // solve's own column pass (p->ws.g, refinement corrections included)
  BndArgs bres{};    // the bounds at the current iterate
  if (bnd) {
    bres.ub = p->ub; bres.s = p->bs; bres.w = p->bw; bres.q = p->bq; bres.ru = p->bru;
  }
  auto resid_stage = [&](bool full) -> ahlp_status_t {
    p->timer.begin(AHLP_ST_RESID);
    const double* zr = z;   // r_d = c - A'y - z (+ w)
    if (bnd) {
      launch_bnd_prep(st, n, p->ub, x, z, p->bs, p->bw, p->bru, p->bq, p->bzw, p->info);
      p->qcur = p->bq;
      zr = p->bzw;
    }
    CHK(prep_scaling(p, x, z, o->rho, st));
    if (bnd) launch_bnd_prep(st, n, p->ub, x, z, p->bs, p->bw, p->bru, p->bq, p->bzw, p->info);
    if (full) apply_At_both(p, y, p->c, zr, p->rd, p->aty, st);
    else launch_rd(st, n, p->c, p->aty, zr, p->rd);
    // rz_a = -x z, rhx_a, vx = D rhx_a, w1 = D / x (- D / s), xp = x (padded);
    // with bounds also the predictor's x right-hand side brdt
    launch_resid_prep(st, p->blk, p->N, p->n0, p->x0off, p->d0off, x, z, p->rd, p->xs, p->Dp,
                      p->rzv, p->ws.rhx, p->ws.vx, p->w1p, p->ws.xp, bres, p->brdt);
    {
      RowsArgs ra{};
      ra.nv = 3;
      ra.v[0] = p->ws.xp; ra.base[0] = p->b; ra.alpha[0] = -1.0; ra.out[0] = p->rp; ra.with_C[0] = 1;
      ra.v[1] = p->ws.vx; ra.alpha[1] = 1.0; ra.out[1] = p->ta; ra.padded[1] = 1; ra.chain[1] = 1;
      ra.v[2] = p->w1p; ra.alpha[2] = 1.0; ra.out[2] = p->aw1; ra.padded[2] = 1;
      rows_pass(p, ra, st);
    }
    link_global_rows(p, p->ws.xp, p->ws.xp + p->d0off, p->b + p->mblk, -1.0, p->rp + p->mblk, st);
    Reds Rr(p);
    Rr.add(RED_DOT, n, x, z, 0).add(RED_DOT, n, p->c, x, 1).add(RED_DOT, m, p->b, y, 2)
        .add(RED_MAXABS, m, p->rp, nullptr, 3).add(RED_MAXABS, n, p->rd, nullptr, 4)
        .add(RED_MAXSUM, n, x, z, 5);
    if (bnd)
      Rr.add(RED_DOT, n, p->bs, p->bw, S_SW).add(RED_MAXABS, n, p->bru, nullptr, S_RU)
          .add(RED_DOT, n, p->ufin, p->bw, S_UW).add(RED_MAXABS, n, p->bq, nullptr, S_QMAX);
    Rr.launch(st);
    p->timer.end();
    return AHLP_OK;
  };
  // the step with the ratio-test results on the device, then the next
  // iteration's residuals
  auto step_resid = [&]() -> ahlp_status_t {
    launch_steps(st, o->eta, StepSet{bnd ? 6 : 4, {n, m, n, n, n, n},
                                     {p->ws.scal + S_AP, p->ws.scal + S_AD, p->ws.scal + S_AD,
                                      p->ws.scal + S_AD, p->ws.scal + S_AP, p->ws.scal + S_AD},
                                     {p->dx, p->dy, p->dz, p->ws.g, p->bds, p->bdw},
                                     {x, y, z, p->aty, p->bs, p->bw}});
    return resid_stage(false);
  };
  CHK(resid_stage(true));
  while (true) {
    CHK(read_scal(p, NSCAL, st));
    if (hinfo->nonfinite & 2)
      return fail(AHLP_EHIP, "the fused factorization launch gave up waiting for its own stages");
    if (hinfo->nonfinite)
      return fail(AHLP_ENUMERIC, "x or z left the positive orthant or became non-finite");
    const double knorm_iter = std::max(p->colabs1_max + (bnd ? hs[S_QMAX] : 0.0),
                                       std::max(p->rowabs_max, hs[5]));
    const long long nmu = n + p->nU;   // complementarity pairs
    mu = (hs[0] + (bnd ? hs[S_SW] : 0.0)) / (double)nmu;
    pobj = hs[1];
    dobj = hs[2] - (bnd ? hs[S_UW] : 0.0);
    relgap = std::fabs(pobj - dobj) / std::max(1.0, std::fabs(pobj));
    pinf = hs[3] / bn;
    if (bnd) pinf = std::max(pinf, hs[S_RU] / (1.0 + p->ub_inf));
    dinf = hs[4] / cn;
    if (o->verbose)
      fprintf(stderr, "ahlp it %3d mu %.3e gap %.3e pinf %.3e dinf %.3e pobj %.10e%s\n", k, mu,
              relgap, pinf, dinf, pobj, fp32_live ? " fp32" : "");
    if (relgap <= o->tol && pinf <= o->tol && dinf <= o->tol) {
      status = AHLP_OK;
      break;
    }
    if (k >= o->max_iter) break;
    if (fp32_live && mu < o->mu_switch) fp32_live = false;
    const double kn = knorm_iter;
    ahlp_ipm_iter_t it;
    std::memset(&it, 0, sizeof it);
    it.mu = mu;

    // One predictor-corrector pass with FP64 or FP32 factors.  A direction is
    // accepted at backward error <= refine_tol; with FP32 factors also at
    // |r - K d| <= fp32_accept * mu (inexact Newton).  Otherwise it is refined;
    // FP32 refinement that stagnates or runs out sets *ok = false.
    auto pass = [&](bool f32, bool* ok) -> ahlp_status_t {
      *ok = true;
      const int prec = f32 ? AHLP_FP32_REFINE : AHLP_FP64;
      if (prec == AHLP_FP32_REFINE) CHK(ensure_fp32(p, st));   // allocates: before any capture
      // fp32_accept < 0: the plain refinement rule for FP32 factors too
      // (backward error <= refine_tol or max_refine corrections, then the
      // last direction is kept, as with FP64 factors)
      const bool plain = f32 && o->fp32_accept < 0.0;
      const double atol = (f32 && !plain) ? o->fp32_accept * mu : 0.0;
      auto acceptable = [&](double b) {
        return b <= o->refine_tol || (atol > 0.0 && check_en(p) <= atol);
      };
      double be = 0.0;
      int steps = 0;
      auto muaff_launch = [&]() {
        Reds Rm(p);
        Rm.add(RED_MUAFF, n, x, p->dxa, S_MUAFF, z, p->dza);
        Rm.m.r[0].ps1 = p->ws.scal + S_AP;
        Rm.m.r[0].ps2 = p->ws.scal + S_AD;
        if (bnd) {
          Rm.add(RED_MUAFF, n, p->bs, p->bdsa, S_MUAFF_SW, p->bw, p->bdwa);
          Rm.m.r[1].ps1 = p->ws.scal + S_AP;
          Rm.m.r[1].ps2 = p->ws.scal + S_AD;
        }
        Rm.launch(st);
      };
      // ratio tests over (x, s) and (z, w)
      auto ratios = [&](Reds& Rq, const double* ddx, const double* ddz, const double* dds,
                        const double* ddw) {
        if (bnd)
          Rq.add(RED_RATIO2, n, x, ddx, S_AP, p->bs, dds).add(RED_RATIO2, n, z, ddz, S_AD, p->bw, ddw);
        else
          Rq.add(RED_RATIO, n, x, ddx, S_AP).add(RED_RATIO, n, z, ddz, S_AD);
      };
      // the bounds' recovery of ds, dw in the checks (predictor, corrector)
      BndArgs bpred = bres, bcorr = bres;
      const double* rxa = p->rd;    // x right-hand sides of predictor and corrector
      const double* rxc = p->rd;
      if (bnd) {
        bpred.mode = 0; bpred.ds = p->bdsa; bpred.dw = p->bdwa;
        bcorr.mode = 1; bcorr.ds = p->bds; bcorr.dw = p->bdw; bcorr.dsa = p->bdsa; bcorr.dwa = p->bdwa;
        bcorr.smu = p->ws.scal + S_SMU; bcorr.rdt = p->brdt;
        rxa = p->brdt;
        rxc = p->brxc;
      }
      const BndArgs* bp = bnd ? &bpred : nullptr;
      const BndArgs* bc = bnd ? &bcorr : nullptr;
      // factorization and predictor (rz_a = -x z; t_a from the residual pass),
      // its check, step lengths and mu_aff
      CHK(run_segment(p, f32 ? SEG_A32 : SEG_A64, key, st, [&]() -> ahlp_status_t {
        CHK(do_factor(p, x, z, prec, o->rho, o->delta, st, true));
        launch_rz(st, n, 0, x, z, nullptr, nullptr, 0.0, p->rzv);
        CHK(solve_once(p, rxa, p->rp, p->rzv, p->dxa, p->dya, p->dza, st, p->ta));
        check_pass(p, rxa, p->rp, p->rzv, p->dxa, p->dza, true, st, bp);
        Reds Rp(p);
        add_check_reds(p, Rp, rxa, p->rp, p->rzv, p->dxa, p->dya, p->dza, true);
        ratios(Rp, p->dxa, p->dza, p->bdsa, p->bdwa);
        Rp.launch(st);
        muaff_launch();
        return AHLP_OK;
      }));
      p->rho = o->rho;
      p->delta = o->delta;
      p->fprec = prec;
      p->factored = true;
      CHK(read_scal(p, NSCAL, st));
      double rn = check_rn(p);
      be = check_bkerr(p, kn, rn);
      if (!acceptable(be)) {
        CHK(refine(p, rxa, p->rp, p->rzv, p->dxa, p->dya, p->dza, o->max_refine, o->refine_tol,
                   kn, rn, true, &be, &steps, st, atol, f32 && !plain, bp));
        if (f32 && !plain && !acceptable(be)) {
          refine_total += steps;   // spent, although the pass is redone in FP64
          *ok = false;
          return AHLP_OK;
        }
        Reds Rq(p);
        ratios(Rq, p->dxa, p->dza, p->bdsa, p->bdwa);
        Rq.launch(st);
        muaff_launch();
        CHK(read_scal(p, NSCAL, st));
      }
      account(be, steps);
      it.bkerr_pred = be;
      it.refine_pred = steps;
      if (o->verbose > 1) fprintf(stderr, "ahlp   predictor bkerr %.2e refine %d\n", be, steps);
      // corrector: sigma mu on the device, rz_c and
      // t_c = t_a - sigma mu A(D/x) + A(D dxa dza / x), solve, check, step lengths
      CHK(run_segment(p, f32 ? SEG_B32 : SEG_B64, key, st, [&]() -> ahlp_status_t {
        if (bnd) launch_sigma_mu(st, p->ws.scal, n + p->nU, 0, S_MUAFF, S_SMU, S_SW, S_MUAFF_SW);
        else launch_sigma_mu(st, p->ws.scal, n, 0, S_MUAFF, S_SMU);
        launch_rz(st, n, 1, x, z, p->dxa, p->dza, 0.0, p->rzv, p->ws.scal + S_SMU, bc,
                  bnd ? p->brxc : nullptr);
        launch_combine(st, p->vp_total, p->ta, 0.0, p->aw1, p->aw2, p->tc, p->ws.scal + S_SMU);
        CHK(solve_once(p, rxc, p->rp, p->rzv, p->dx, p->dy, p->dz, st, p->tc));
        check_pass(p, rxc, p->rp, p->rzv, p->dx, p->dz, false, st, bc);
        Reds Rc(p);
        add_check_reds(p, Rc, rxc, p->rp, p->rzv, p->dx, p->dy, p->dz, true);
        ratios(Rc, p->dx, p->dz, p->bds, p->bdw);
        Rc.launch(st);
        return AHLP_OK;
      }));
      CHK(read_scal(p, NSCAL, st));
      rn = check_rn(p);
      be = check_bkerr(p, kn, rn);
      steps = 0;
      if (!acceptable(be)) {
        CHK(refine(p, rxc, p->rp, p->rzv, p->dx, p->dy, p->dz, o->max_refine, o->refine_tol, kn,
                   rn, false, &be, &steps, st, atol, f32 && !plain, bc));
        if (f32 && !plain && !acceptable(be)) {
          refine_total += steps;   // spent, although the pass is redone in FP64
          *ok = false;
          return AHLP_OK;
        }
        Reds Rq(p);
        ratios(Rq, p->dx, p->dz, p->bds, p->bdw);
        Rq.launch(st);
        CHK(read_scal(p, NSCAL, st));
      }
      account(be, steps);
      it.bkerr_corr = be;
      it.refine_corr = steps;
      it.sigma = hs[S_SMU] / mu;
      if (o->verbose > 1) fprintf(stderr, "ahlp   corrector bkerr %.2e refine %d\n", be, steps);
      return AHLP_OK;
    };
    bool ok = false;
    if (fp32_live) {
      CHK(pass(true, &ok));
      if (ok) {
        R.fp32_iterations++;
        it.fp32 = 1;
      } else {
        // FP32 factors cannot deliver acceptable directions any more: FP64
        // factors from here on, and this iteration is redone with them
        fp32_live = false;
        if (o->verbose) fprintf(stderr, "ahlp   FP32 refinement stalled: FP64 from here\n");
      }
    }
    if (!ok) CHK(pass(false, &ok));
    total_piv += hinfo->pivots;
    // the same step lengths as the step kernels take on the device
    double ap = std::min(1.0, o->eta * hs[S_AP]);
    double ad = std::min(1.0, o->eta * hs[S_AD]);
    // Gondzio's multiple centrality correctors: aim for step lengths longer by
    // delta_a, move the complementarity products at that trial point into
    // [beta_min, beta_max] sigma mu, solve with right-hand side (0, 0, t - v)
    // and keep the corrected direction if the smaller step grows by at least
    // gamma delta_a (constants as in the oracle)
    // g = A'dy of the direction taken, for the A'y update: each correction
    // solve leaves its own A'dy_c in p->ws.g, so the sum is kept in p->gdir
    bool gz_used = false;
    for (int j = 0; j < o->gondzio; ++j) {
      if (ap >= 1.0 && ad >= 1.0) break;
      if (!gz_used) {
        launch_copy(st, n, p->ws.g, p->gdir);
        gz_used = true;
      }
      constexpr double beta_min = 0.1, beta_max = 10.0, delta_a = 0.1, gamma = 0.1;
      const double at_p = std::min(1.0, ap + delta_a), at_d = std::min(1.0, ad + delta_a);
      launch_gondzio_rhs(st, n, x, z, p->dx, p->dz, at_p, at_d, p->ws.scal + S_SMU, beta_min,
                         beta_max, p->g_r);
      double gbe = 0.0;
      int gsteps = 0;
      CHK(solve_refined(p, p->zerosn, p->zerosm, p->g_r, p->g_dx, p->g_dy, p->g_dz,
                        o->max_refine, o->refine_tol, kn, &gbe, &gsteps, st));
      account(gbe, gsteps);
      launch_axpy(st, n, 1.0, p->dx, p->g_dx);
      launch_axpy(st, m, 1.0, p->dy, p->g_dy);
      launch_axpy(st, n, 1.0, p->dz, p->g_dz);
      Reds(p).add(RED_RATIO, n, x, p->g_dx, S_GP).add(RED_RATIO, n, z, p->g_dz, S_GD).launch(st);
      CHK(read_scal(p, NSCAL, st));
      const double ap_n = std::min(1.0, o->eta * hs[S_GP]);
      const double ad_n = std::min(1.0, o->eta * hs[S_GD]);
      if (!(std::min(ap_n, ad_n) >= std::min(ap, ad) + gamma * delta_a)) break;
      launch_copy(st, n, p->g_dx, p->dx);
      launch_copy(st, m, p->g_dy, p->dy);
      launch_copy(st, n, p->g_dz, p->dz);
      launch_copy(st, 2, p->ws.scal + S_GP, p->ws.scal + S_AP);   // the step kernels read S_AP, S_AD
      launch_axpy(st, n, 1.0, p->ws.g, p->gdir);
      ap = ap_n;
      ad = ad_n;
      R.correctors++;
      it.correctors++;
    }
    if (gz_used) launch_copy(st, n, p->gdir, p->ws.g);
    it.alpha_p = ap;
    it.alpha_d = ad;
    p->hist.push_back(it);
    ++k;
    if (ap < 1e-12 && ad < 1e-12) {
      launch_steps(st, o->eta, StepSet{bnd ? 5 : 3, {n, m, n, n, n, 0},
                                       {p->ws.scal + S_AP, p->ws.scal + S_AD, p->ws.scal + S_AD,
                                        p->ws.scal + S_AP, p->ws.scal + S_AD, nullptr},
                                       {p->dx, p->dy, p->dz, p->bds, p->bdw, nullptr},
                                       {x, y, z, p->bs, p->bw, nullptr}});
      status = AHLP_WSTALL;
      break;
    }
    CHK(run_segment(p, SEG_C, key, st, step_resid));
  }
  HIPCHK(hipStreamSynchronize(st));
  p->timer.collect();
  R.status = status;
  R.iterations = k;
  R.refine_steps = refine_total;
  R.pivots_modified = total_piv;
  R.primal_obj = pobj;
  R.dual_obj = dobj;
  R.rel_gap = relgap;
  R.rel_pinf = pinf;
  R.rel_dinf = dinf;
  R.mu = mu;
  R.max_bkerr = max_bk;
  for (int i = 0; i < AHLP_ST_COUNT; ++i) {
    R.t_stage_ms[i] = p->timer.ms[i];
    R.n_stage[i] = p->timer.cnt[i];
    R.t_stage32_ms[i] = p->timer.ms32[i];
    R.n_stage32[i] = p->timer.cnt32[i];
  }
  R.rows_bytes = p->rows_bytes;
  p->timer.on = false;
  R.t_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (res) *res = R;
  return status;
}

ahlp_status_t ahlp_ipm_history(ahlp_problem_t p, ahlp_ipm_iter_t* out, int32_t cap,
                               int32_t* count) {
  g_err.clear();
  if (!p || !count) return fail(AHLP_EINVAL, "null argument");
  if (cap < 0 || (cap > 0 && !out)) return fail(AHLP_EINVAL, "need cap >= 0 and out for cap > 0");
  *count = (int32_t)p->hist.size();
  const int32_t w = std::min<int32_t>(cap, *count);
  for (int32_t i = 0; i < w; ++i) out[i] = p->hist[i];
  return AHLP_OK;
}

// ---------------------------------------------------------------- inspection
ahlp_status_t ahlp_problem_sizes(ahlp_problem_t p, int64_t* n_tot, int64_t* m_tot,
                                 int64_t* n_link, int32_t* n0) {
  if (!p) return fail(AHLP_EINVAL, "null handle");
  if (n_tot) *n_tot = p->n_tot;
  if (m_tot) *m_tot = p->m_tot;
  if (n_link) *n_link = p->nl;
  if (n0) *n0 = p->n0;
  return AHLP_OK;
}

// Device ceilings: one untimed launch, then the best of three timed ones.
namespace {
struct CeilBuf {
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~CeilBuf() {
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};
ahlp_status_t ceil_grid(int per_cu, int* grid) {
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *grid = std::max(cus, 1) * per_cu;
  return AHLP_OK;
}
}  // namespace

ahlp_status_t ahlp_ceiling_mfma(int32_t precision, double* tflops, hipStream_t stream) {
  if (!tflops) return fail(AHLP_EINVAL, "null argument");
  if (precision != AHLP_FP64 && precision != AHLP_FP32_REFINE)
    return fail(AHLP_EINVAL, "unknown precision %d", precision);
  const bool f32 = precision == AHLP_FP32_REFINE;
  int grid = 0;
  CHK(ceil_grid(8, &grid));   // eight four-wave workgroups per CU: eight waves per SIMD
  const int iters = f32 ? 2048 : 1024;   // multiples of the kernel's sixteen rounds per trip
  CeilBuf cb;
  HIPCHK(hipMalloc(&cb.out, (size_t)grid * sizeof(double)));
  HIPCHK(hipEventCreate(&cb.e0));
  HIPCHK(hipEventCreate(&cb.e1));
  launch_ceiling_mfma(stream, f32, grid, iters, cb.out);
  float best = 0.f;
  for (int rep = 0; rep < 3; ++rep) {
    HIPCHK(hipEventRecord(cb.e0, stream));
    launch_ceiling_mfma(stream, f32, grid, iters, cb.out);
    HIPCHK(hipEventRecord(cb.e1, stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(cb.e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, cb.e0, cb.e1));
    if (rep == 0 || ms < best) best = ms;
  }
  // per wave and iteration eight 16x16x4 products of 2048 flops
  const double flop = (double)grid * 4 * iters * 8 * 2048.0;
  *tflops = best > 0.f ? flop / (best * 1e-3) / 1e12 : 0.0;
  return AHLP_OK;
}

ahlp_status_t ahlp_ceiling_hbm_read(const double* buf, int64_t n, double* gbps,
                                    hipStream_t stream) {
  if (!buf || !gbps || n < 2 || (reinterpret_cast<uintptr_t>(buf) & 15))
    return fail(AHLP_EINVAL, "null or misaligned buffer, or n < 2");
  int grid = 0;
  CHK(ceil_grid(16, &grid));
  CeilBuf cb;
  HIPCHK(hipMalloc(&cb.out, (size_t)grid * sizeof(double)));
  HIPCHK(hipEventCreate(&cb.e0));
  HIPCHK(hipEventCreate(&cb.e1));
  launch_ceiling_read(stream, buf, n, grid, cb.out);
  float best = 0.f;
  for (int rep = 0; rep < 3; ++rep) {
    HIPCHK(hipEventRecord(cb.e0, stream));
    launch_ceiling_read(stream, buf, n, grid, cb.out);
    HIPCHK(hipEventRecord(cb.e1, stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(cb.e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, cb.e0, cb.e1));
    if (rep == 0 || ms < best) best = ms;
  }
  const double bytes = (double)(n / 2) * 16.0;
  *gbps = best > 0.f ? bytes / (best * 1e-3) / 1e9 : 0.0;
  return AHLP_OK;
}

ahlp_status_t ahlp_ceiling_tile_chol(int32_t beside_mfma, double* us_per_tile,
                                     hipStream_t stream) {
  if (!us_per_tile) return fail(AHLP_EINVAL, "null argument");
  if (beside_mfma != 0 && beside_mfma != 1) return fail(AHLP_EINVAL, "beside_mfma must be 0 or 1");
  int grid = 0;
  CHK(ceil_grid(1, &grid));   // one workgroup per CU
  const int iters = 256;
  CeilBuf cb;
  HIPCHK(hipMalloc(&cb.out, (size_t)grid * sizeof(double)));
  HIPCHK(hipEventCreate(&cb.e0));
  HIPCHK(hipEventCreate(&cb.e1));
  launch_ceiling_chol(stream, beside_mfma == 1, grid, iters, cb.out);
  float best = 0.f;
  for (int rep = 0; rep < 3; ++rep) {
    HIPCHK(hipEventRecord(cb.e0, stream));
    launch_ceiling_chol(stream, beside_mfma == 1, grid, iters, cb.out);
    HIPCHK(hipEventRecord(cb.e1, stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(cb.e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, cb.e0, cb.e1));
    if (rep == 0 || ms < best) best = ms;
  }
  // the launch lasts as long as the factoring waves' loop (the streaming
  // waves stop at its flag)
  *us_per_tile = (double)best * 1e3 / iters;
  return AHLP_OK;
}

ahlp_status_t ahlp_debug_pivots(ahlp_problem_t p, int32_t* count) {
  if (!p || !count) return fail(AHLP_EINVAL, "null argument");
  CHK(check_info(p, p->timer.st, nullptr));
  *count = p->pivots_seen;
  return AHLP_OK;
}

ahlp_status_t ahlp_debug_block(ahlp_problem_t p, int32_t i, double* L, double* W) {
  if (!p || i < 0 || i >= p->N) return fail(AHLP_EINVAL, "bad block index");
  if (!p->factored) return fail(AHLP_ESTATE, "no factorization");
  const BlockInfo& b = p->hb[i];
  const long long ntile = lb_tiles(b.mt, b.rt) * 256;
  std::vector<double> h((size_t)ntile);
  HIPCHK(hipDeviceSynchronize());
  if (p->fprec == AHLP_FP32_REFINE) {
    std::vector<float> hf((size_t)ntile);
    HIPCHK(hipMemcpy(hf.data(), p->LB32 + b.lboff, sizeof(float) * ntile, hipMemcpyDeviceToHost));
    for (long long t = 0; t < ntile; ++t) h[t] = hf[t];
  } else {
    HIPCHK(hipMemcpy(h.data(), p->LB + b.lboff, sizeof(double) * ntile, hipMemcpyDeviceToHost));
  }
  auto at = [&](int r, int c) {  // element (r, c) of the bordered factor, r >= c
    BlockInfo b0 = b;
    b0.lboff = 0;
    return h[lb_tile(b0, r / 16, c / 16) + (c % 16) * 16 + r % 16];
  };
  if (L) {
    for (int r = 0; r < b.m; ++r)
      for (int c = 0; c < b.m; ++c) L[(long long)r * b.m + c] = (c <= r) ? at(r, c) : 0.0;
  }
  if (W) {
    const int k = b.lL + b.lR + p->nb;
    for (int a = 0; a < b.m; ++a)
      for (int col = 0; col < k; ++col) {
        int q;
        if (col < b.lL) q = col;
        else if (col < b.lL + b.lR) q = 16 * b.ktL + (col - b.lL);
        else q = 16 * (b.ktL + b.ktR) + (col - b.lL - b.lR);
        W[(long long)a * k + col] = at(16 * b.mt + q, a);
      }
  }
  return AHLP_OK;
}

ahlp_status_t ahlp_debug_schur(ahlp_problem_t p, double* S) {
  if (!p || !S) return fail(AHLP_EINVAL, "null argument");
  if (!p->factored) return fail(AHLP_ESTATE, "no factorization");
  const long long dim = p->nl + p->nb;
  HIPCHK(hipDeviceSynchronize());
  std::vector<double> Td, To, E, S00;
  auto fetch = [&](std::vector<double>& v, const double* src, long long cnt) -> ahlp_status_t {
    v.resize((size_t)std::max(cnt, 1LL));
    if (cnt > 0) HIPCHK(hipMemcpy(v.data(), src, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    return AHLP_OK;
  };
  const int P = p->P, n0 = p->nb;   // the border: global rows, then x_0
  long long tdn = P > 0 ? p->tdoff[P - 1] + (long long)p->l[P - 1] * p->l[P - 1] : 0;
  long long ton = P > 1 ? p->tooff[P - 2] + (long long)p->l[P - 1] * p->l[P - 2] : 0;
  CHK(fetch(Td, p->Td, tdn));
  CHK(fetch(To, p->To, ton));
  CHK(fetch(E, p->E, p->nl * n0));
  CHK(fetch(S00, p->S00, (long long)n0 * n0));
  std::fill(S, S + dim * dim, 0.0);
  for (int j = 0; j < P; ++j) {
    const int l = p->l[j];
    const long long o = p->loff[j];
    for (int a = 0; a < l; ++a)
      for (int c = 0; c < l; ++c) S[(o + a) * dim + o + c] = Td[p->tdoff[j] + a + (long long)c * l];
    if (j + 1 < P) {
      const int l2 = p->l[j + 1];
      const long long o2 = p->loff[j + 1];
      for (int a = 0; a < l2; ++a)
        for (int c = 0; c < l; ++c) {
          const double v = To[p->tooff[j] + a + (long long)c * l2];
          S[(o2 + a) * dim + o + c] = v;
          S[(o + c) * dim + o2 + a] = v;
        }
    }
    for (int a = 0; a < l; ++a)
      for (int c = 0; c < n0; ++c) {
        const double v = E[p->eoff[j] + a + (long long)c * l];
        S[(o + a) * dim + p->nl + c] = v;
        S[(p->nl + c) * dim + o + a] = v;
      }
  }
  for (int a = 0; a < n0; ++a)
    for (int c = 0; c < n0; ++c) S[(p->nl + a) * dim + p->nl + c] = S00[a + (long long)c * n0];
  return AHLP_OK;
}

}  // extern "C"
