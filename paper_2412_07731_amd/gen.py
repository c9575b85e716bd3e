"""Seeded synthetic arrowhead LPs with a known optimum.

This module only draws problem data; it contains none of the interior-point
method's arithmetic, so both the GPU path and the CPU oracle may use it.

The LP is the standard-form problem of Sec. 2.2 (min c'x, Ax = b, x >= 0) with
the arrowhead block structure of Sec. 3.2, restricted to equality rows,
x >= 0 bounds and local (two-link) linking constraints (Sec. 3.3):

    block rows   A_i x_i + C_i x_0                   = b_i      i = 1..N
    link rows    FR_j x_j + FL_j x_{j+1} + F0_j x_0  = b_Lj     j = 1..N-1
    global rows  Wg_1 x_1 + ... + Wg_N x_N + Wg_0 x_0 = b_G     (optional)

Here ``A_i`` is the paper's B_i, ``C_i`` the paper's A_i (coupling to the
linking variables x_0), ``FR_j`` the paper's local block F_j and ``FL_j`` the
paper's F'_j; ``Wg_i`` are the global linking rows (the paper's F with
global support, Sec. 3.3).  Canonical vector order: x = [x_1..x_N, x_0],
y = [y_1..y_N, y_L, y_G] with y_L listing the link pairs in order.

Known optimum (complementary primal/dual pair chosen first, data derived):
  * x*: in every block exactly floor(n_i/2) entries ~U[0.5, 2], the rest 0;
    the same for x_0 with floor(n0/2);
  * z*: ~U[0.5, 2] where x* = 0, else 0;  y* ~ N(0, 1);
  * b = A x*,  c = A' y* + z*,  so f* = c'x* = b'y*.

Storage-continuity links: row k of pair j has +1 on variable n_j - l_j + k of
block j and -1 on variable k of block j+1 (energy-system storage balance).

Draw order (fixed; PCG64(seed)): random sizes (m_i, then l_j), then per block
A_i (mask, values, zero-row redraws) and C_i (mask, values), then (only with
ng > 0 global rows) per block and row three distinct columns and their values
~U[-1, 1], and Wg_0 (mask, values), then x* positions and values per block and
for x_0, then z* values, then y*, then (only with ub_frac > 0) the bounded
mask, the at-bound mask, the slacks of the inactive bounds and the duals w* of
the active ones, one draw of each per variable.

Nondegenerate variant (``nondegenerate=True``, needs n0 = 0), for the
sensitivity workload: block i gets exactly m_i + l_i positive x* entries (l_i
of the pair on its right, 0 for the last block): its last l_i variables (the
pair's boundary variables, forced in) and m_i others drawn from the variables
that touch no link row (not the first l_{i-1}, not the last l_i), redrawn
until A_i restricted to them is nonsingular.  The basis matrix A_B is then
block diagonal with blocks [[A_i(:, R_i), A_i(:, bd_i)], [0, I]], so it is
square and nonsingular, x*_B > 0 and z*_N > 0: the optimum is unique and
strictly complementary.  Draws: the m_i others (and redraws) then the x*_B
values per block, then z* values, then y*.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Named workload shapes (time-block LPs shaped like the paper's energy-system
# models; see the experiments of Sec. 5 for the structure they stand in for).
CONFIGS = {
    # tiny: N=8, 32x64 blocks at 30% density, 4 links per pair, 8 linking vars
    "tiny": dict(N=8, m=32, n=64, l=4, n0=8, density=0.30),
    # full size: N=512, 256x512 blocks at 10%, 16 links per pair, 32 linking vars
    "n512": dict(N=512, m=256, n=512, l=16, n0=32, density=0.10),
    # uneven blocks: m_i ~ U{64..512}, n_i = 2 m_i, l_j ~ U{4..32}, 64 linking vars
    "uneven": dict(N=2048, m=(64, 512), n="2m", l=(4, 32), n0=64, density=0.10),
    # sensitivity workload: N=256, 256x512 at 10%, 16 links, no linking vars,
    # nondegenerate optimum
    "sens": dict(N=256, m=256, n=512, l=16, n0=0, density=0.10, nondegenerate=True),
    # small nondegenerate instance for dense reference checks
    "tiny_nd": dict(N=8, m=32, n=64, l=4, n0=0, density=0.30, nondegenerate=True),
    # global linking rows kept whole (each touches every block and x_0): tiny
    # with 3 of them, and a mid-size case with 20 (a border of 20 + 16 rows)
    "tiny_g": dict(N=8, m=32, n=64, l=4, n0=8, density=0.30, ng=3),
    "mid_g": dict(N=40, m=48, n=96, l=16, n0=16, density=0.10, ng=20),
    # upper bounds on 40% of the variables (0 <= x <= u), some active at the
    # optimum: tiny, and 64 blocks of 96x192
    "tiny_b": dict(N=8, m=32, n=64, l=4, n0=8, density=0.30, ub_frac=0.4),
    "mid_b": dict(N=64, m=96, n=192, l=8, n0=16, density=0.10, ub_frac=0.4),
}


@dataclass
class Instance:
    """An arrowhead LP in the block form above (all arrays float64, row-major)."""

    N: int
    n0: int
    m: np.ndarray                 # int64 [N]
    n: np.ndarray                 # int64 [N]
    l: np.ndarray                 # int64 [N-1]
    A: List[np.ndarray]           # m_i x n_i
    C: List[np.ndarray]           # m_i x n0
    FR: List[np.ndarray]          # pair j: l_j x n_j      (block j's part)
    FL: List[np.ndarray]          # pair j: l_j x n_{j+1}  (block j+1's part)
    F0: Optional[np.ndarray]      # (sum l) x n0, or None for zero
    b: np.ndarray                 # [block rows, link rows, global rows]
    c: np.ndarray
    Wg: Optional[List[np.ndarray]] = field(default=None)   # global rows: ng x n_i per block
    Wg0: Optional[np.ndarray] = field(default=None)        # their x_0 part, ng x n0
    ub: Optional[np.ndarray] = field(default=None)         # upper bounds [n_tot] (inf: none)
    xstar: np.ndarray = field(default=None)
    ystar: np.ndarray = field(default=None)
    zstar: np.ndarray = field(default=None)
    fstar: float = float("nan")
    basis: Optional[list] = field(default=None)   # nondegenerate variant: positive x* indices per block

    @property
    def ng(self) -> int:
        """Global linking rows (each over every block and x_0)."""
        return 0 if self.Wg is None else int(self.Wg[0].shape[0])

    @property
    def n_tot(self) -> int:
        return int(self.n.sum()) + self.n0

    @property
    def m_tot(self) -> int:
        return int(self.m.sum()) + int(self.l.sum()) + self.ng

    def xoff(self) -> np.ndarray:
        """Start of each block's variables in x (length N+1; last = x_0 start)."""
        return np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)

    def yoff(self) -> np.ndarray:
        """Start of each block's rows in y (length N+1; last = y_L start)."""
        return np.concatenate([[0], np.cumsum(self.m)]).astype(np.int64)

    def loff(self) -> np.ndarray:
        """Start of each link pair inside y_L (length N)."""
        return np.concatenate([[0], np.cumsum(self.l)]).astype(np.int64)


def _sizes(cfg, rng):
    N = cfg["N"]
    m = cfg["m"]
    if isinstance(m, tuple):
        m = rng.integers(m[0], m[1] + 1, size=N)
    else:
        m = np.full(N, m)
    n = cfg["n"]
    if n == "2m":
        n = 2 * m
    else:
        n = np.full(N, n)
    l = cfg["l"]
    if isinstance(l, tuple):
        l = rng.integers(l[0], l[1] + 1, size=max(N - 1, 0))
    else:
        l = np.full(max(N - 1, 0), l)
    m = np.asarray(m, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    l = np.asarray(l, dtype=np.int64)
    for j in range(N - 1):
        if l[j] > min(n[j], n[j + 1]):
            raise ValueError("link pair larger than a neighbouring block")
    return m, n, l


def _sparse_block(rng, rows, cols, density, redraw_zero_rows):
    mask = rng.random((rows, cols)) < density
    vals = rng.uniform(-1.0, 1.0, size=(rows, cols))
    X = np.where(mask, vals, 0.0)
    if redraw_zero_rows and cols > 0:
        while True:
            zero = np.flatnonzero(~X.any(axis=1))
            if zero.size == 0:
                break
            mask = rng.random((zero.size, cols)) < density
            vals = rng.uniform(-1.0, 1.0, size=(zero.size, cols))
            X[zero] = np.where(mask, vals, 0.0)
    return X


def generate(config="tiny", seed=0, **overrides) -> Instance:
    """Draw one instance.  ``config`` is a name from CONFIGS or a dict."""
    cfg = dict(CONFIGS[config]) if isinstance(config, str) else dict(config)
    cfg.update(overrides)
    rng = np.random.Generator(np.random.PCG64(seed))
    N, n0, dens = int(cfg["N"]), int(cfg["n0"]), float(cfg["density"])
    m, n, l = _sizes(cfg, rng)

    A, C = [], []
    for i in range(N):
        A.append(_sparse_block(rng, int(m[i]), int(n[i]), dens, True))
        C.append(_sparse_block(rng, int(m[i]), n0, dens, False))

    FR, FL = [], []
    for j in range(N - 1):
        lj = int(l[j])
        fr = np.zeros((lj, int(n[j])))
        fl = np.zeros((lj, int(n[j + 1])))
        for k in range(lj):
            fr[k, int(n[j]) - lj + k] = 1.0
            fl[k, k] = -1.0
        FR.append(fr)
        FL.append(fl)
    F0 = None

    # global rows: three random entries per row in every block, ~U[-1, 1],
    # and the x_0 part at the block density
    ng = int(cfg.get("ng", 0))
    Wg = Wg0 = None
    if ng > 0:
        Wg = []
        for i in range(N):
            W = np.zeros((ng, int(n[i])))
            for k in range(ng):
                cols = rng.choice(int(n[i]), size=min(3, int(n[i])), replace=False)
                W[k, cols] = rng.uniform(-1.0, 1.0, size=cols.size)
            Wg.append(W)
        Wg0 = _sparse_block(rng, ng, n0, dens, False)

    # complementary optimum
    xs = []
    basis = None
    if cfg.get("nondegenerate", False):
        if n0 != 0:
            raise ValueError("the nondegenerate variant needs n0 = 0")
        basis = []
        for i in range(N):
            ni, mi = int(n[i]), int(m[i])
            lr = int(l[i]) if i < N - 1 else 0
            ll = int(l[i - 1]) if i > 0 else 0
            pool = np.arange(ll, ni - lr)
            if pool.size < mi:
                raise ValueError("block too narrow for a nondegenerate basis")
            while True:
                R = np.sort(rng.choice(pool, size=mi, replace=False))
                if np.linalg.matrix_rank(A[i][:, R]) == mi:
                    break
            Bi = np.concatenate([R, np.arange(ni - lr, ni)])
            xi = np.zeros(ni)
            xi[Bi] = rng.uniform(0.5, 2.0, size=Bi.size)
            xs.append(xi)
            basis.append(Bi)
        xs.append(np.zeros(0))
    else:
        for i in range(N + 1):
            ni = int(n[i]) if i < N else n0
            xi = np.zeros(ni)
            pos = rng.permutation(ni)[: ni // 2]
            xi[pos] = rng.uniform(0.5, 2.0, size=pos.size)
            xs.append(xi)
    xstar = np.concatenate(xs) if xs else np.zeros(0)
    zvals = rng.uniform(0.5, 2.0, size=xstar.size)
    zstar = np.where(xstar == 0.0, zvals, 0.0)
    m_tot = int(m.sum() + l.sum()) + ng
    ystar = rng.standard_normal(m_tot)

    # upper bounds (only with ub_frac > 0): a variable is bounded with
    # probability ub_frac; a bounded positive x*_j is at its bound with
    # probability 1/2 (u = x*, dual w* ~U[0.5, 2]), else u = x* + ~U[0.5, 2]
    ub = wstar = None
    frac = float(cfg.get("ub_frac", 0.0))
    if frac > 0.0:
        nt = xstar.size
        bmask = rng.random(nt) < frac
        at = (rng.random(nt) < 0.5) & (xstar > 0.0)
        slack = rng.uniform(0.5, 2.0, size=nt)
        wv = rng.uniform(0.5, 2.0, size=nt)
        ub = np.where(bmask, np.where(at, xstar, xstar + slack), np.inf)
        wstar = np.where(bmask & at, wv, 0.0)

    inst = Instance(N=N, n0=n0, m=m, n=n, l=l, A=A, C=C, FR=FR, FL=FL, F0=F0,
                    b=np.zeros(m_tot), c=np.zeros(xstar.size), Wg=Wg, Wg0=Wg0, ub=ub)
    inst.xstar, inst.ystar, inst.zstar = xstar, ystar, zstar
    inst.basis = basis   # per block: the indices of the positive x* entries (nondegenerate only)
    inst.b = apply_A(inst, xstar)
    inst.c = apply_At(inst, ystar) + zstar
    if wstar is not None:
        inst.c = inst.c - wstar      # dual of the active upper bounds: A'y* + z* - w* = c
        inst.wstar = wstar
    inst.fstar = float(inst.c @ xstar)
    return inst


# The two products below define the data b and c from the chosen optimum; they
# are the LP's constraint operator written out block by block.

def apply_A(inst: Instance, x: np.ndarray) -> np.ndarray:
    xo, yo, lo = inst.xoff(), inst.yoff(), inst.loff()
    x0 = x[xo[-1]:]
    out = np.zeros(inst.m_tot)
    for i in range(inst.N):
        xi = x[xo[i]:xo[i + 1]]
        out[yo[i]:yo[i + 1]] = inst.A[i] @ xi + inst.C[i] @ x0
    base = yo[-1]
    for j in range(inst.N - 1):
        s = slice(base + lo[j], base + lo[j + 1])
        out[s] = inst.FR[j] @ x[xo[j]:xo[j + 1]] + inst.FL[j] @ x[xo[j + 1]:xo[j + 2]]
        if inst.F0 is not None:
            out[s] += inst.F0[lo[j]:lo[j + 1]] @ x0
    base += lo[-1]
    for k in range(inst.ng):
        out[base + k] = sum(inst.Wg[i][k] @ x[xo[i]:xo[i + 1]] for i in range(inst.N))
        if inst.n0:
            out[base + k] += inst.Wg0[k] @ x0
    return out


def apply_At(inst: Instance, y: np.ndarray) -> np.ndarray:
    xo, yo, lo = inst.xoff(), inst.yoff(), inst.loff()
    out = np.zeros(inst.n_tot)
    base = yo[-1]
    x0s = slice(xo[-1], inst.n_tot)
    for i in range(inst.N):
        yi = y[yo[i]:yo[i + 1]]
        out[xo[i]:xo[i + 1]] += inst.A[i].T @ yi
        out[x0s] += inst.C[i].T @ yi
    for j in range(inst.N - 1):
        yl = y[base + lo[j]: base + lo[j + 1]]
        out[xo[j]:xo[j + 1]] += inst.FR[j].T @ yl
        out[xo[j + 1]:xo[j + 2]] += inst.FL[j].T @ yl
        if inst.F0 is not None:
            out[x0s] += inst.F0[lo[j]:lo[j + 1]].T @ yl
    if inst.ng:
        yg = y[base + lo[-1]:]
        for i in range(inst.N):
            out[xo[i]:xo[i + 1]] += inst.Wg[i].T @ yg
        if inst.n0:
            out[x0s] += inst.Wg0.T @ yg
    return out


# --------------------------------------------------------------------------
# General arrowhead form (Sec. 3.2): inequality rows and variable bounds.
#
#   block rows      A_i x_i + C_i x_0                  = b_i
#                   d_i <= H_i x_i + G_i x_0 <= f_i            i = 1..N
#   x_0 rows        d_0 <= G_0 x_0 <= f_0
#   link rows       FR_j x_j + FL_j x_{j+1} (+ F0_j x_0) = b_Lj
#                   dl_j <= KR_j x_j + KL_j x_{j+1} <= fl_j    j = 1..N-1
#   global rows     dg <= Wg_1 x_1 + ... + Wg_N x_N + Wg_0 x_0 <= fg
#                   (an equality where dg = fg)
#   x_0 rows        A_0 x_0 = b_0   (full row rank)
#   bounds          lo <= x <= up   (entries may be -inf / +inf, lo < up)
#
# Inequality sides may be infinite (one side at a time).

@dataclass
class GeneralInstance:
    N: int
    n0: int
    m: np.ndarray                 # equality rows per block [N]
    n: np.ndarray                 # variables per block [N]
    l: np.ndarray                 # equality rows per link pair [N-1]
    A: List[np.ndarray]
    C: List[np.ndarray]
    FR: List[np.ndarray]
    FL: List[np.ndarray]
    F0: Optional[np.ndarray]
    b: np.ndarray                 # [sum m + sum l], block rows then link rows
    H: List[np.ndarray]           # inequality rows of block i: mi_i x n_i
    G: List[np.ndarray]           # and their x_0 part: mi_i x n0
    d: List[np.ndarray]
    f: List[np.ndarray]
    G0: np.ndarray                # x_0-only inequality rows: mi0 x n0
    d0: np.ndarray
    f0: np.ndarray
    KR: List[np.ndarray]          # inequality rows of link pair j: li_j x n_j
    KL: List[np.ndarray]          # li_j x n_{j+1}
    dl: List[np.ndarray]
    fl: List[np.ndarray]
    c: np.ndarray                 # [n_tot], canonical order [x_1..x_N, x_0]
    lo: np.ndarray
    up: np.ndarray
    Wg: List[np.ndarray] = field(default_factory=list)   # global rows, block i part: ng x n_i
    Wg0: Optional[np.ndarray] = None                      # global rows, x_0 part: ng x n0
    dg: np.ndarray = field(default_factory=lambda: np.zeros(0))
    fg: np.ndarray = field(default_factory=lambda: np.zeros(0))
    A0: Optional[np.ndarray] = None                       # x_0-only equality rows: me0 x n0
    b0: np.ndarray = field(default_factory=lambda: np.zeros(0))
    xhat: np.ndarray = field(default=None)   # the interior point the data were drawn around

    @property
    def ng(self) -> int:
        return int(self.dg.size)

    @property
    def n_tot(self) -> int:
        return int(self.n.sum()) + self.n0


def general_matrices(g: GeneralInstance):
    """The constraint rows of a general instance as global sparse matrices
    (columns in canonical order): (Aeq, beq, Ain, lower, upper) with equality
    rows [blocks, links, global equalities, x_0-only] and inequality rows
    [blocks, x_0-only, links, global inequalities]."""
    import scipy.sparse as sp
    xo = np.concatenate([[0], np.cumsum(g.n)]).astype(np.int64)
    nt = g.n_tot

    def place(parts):
        # parts: list of (rows x width dense array, column offset)
        rows = parts[0][0].shape[0]
        M = sp.lil_matrix((rows, nt))
        for X, off in parts:
            if X is not None and X.size:
                M[:, off:off + X.shape[1]] = X
        return M.tocsr()

    eq = []
    for i in range(g.N):
        eq.append(place([(g.A[i], xo[i]), (g.C[i], xo[-1])]))
    lo_ = np.concatenate([[0], np.cumsum(g.l)]).astype(np.int64)
    for j in range(g.N - 1):
        parts = [(g.FR[j], xo[j]), (g.FL[j], xo[j + 1])]
        if g.F0 is not None:
            parts.append((g.F0[lo_[j]:lo_[j + 1]], xo[-1]))
        eq.append(place(parts))
    ineq, lower, upper = [], [], []
    for i in range(g.N):
        ineq.append(place([(g.H[i], xo[i]), (g.G[i], xo[-1])]))
        lower.append(g.d[i]); upper.append(g.f[i])
    ineq.append(place([(g.G0, xo[-1])]))
    lower.append(g.d0); upper.append(g.f0)
    for j in range(g.N - 1):
        ineq.append(place([(g.KR[j], xo[j]), (g.KL[j], xo[j + 1])]))
        lower.append(g.dl[j]); upper.append(g.fl[j])
    beq = [g.b]
    if g.ng:
        Wrow = place([(g.Wg[i], xo[i]) for i in range(g.N)] + [(g.Wg0, xo[-1])])
        is_eq = g.dg == g.fg
        if is_eq.any():
            eq.append(Wrow[np.flatnonzero(is_eq)])
            beq.append(g.dg[is_eq])
        if (~is_eq).any():
            ineq.append(Wrow[np.flatnonzero(~is_eq)])
            lower.append(g.dg[~is_eq]); upper.append(g.fg[~is_eq])
    if g.A0 is not None and g.A0.shape[0]:
        eq.append(place([(g.A0, xo[-1])]))
        beq.append(g.b0)
    Aeq = sp.vstack(eq).tocsr() if eq else sp.csr_matrix((0, nt))
    Ain = sp.vstack(ineq).tocsr()
    return Aeq, np.concatenate(beq), Ain, np.concatenate(lower), np.concatenate(upper)


GENERAL_CONFIGS = {
    # small: every bound and row kind on a few blocks (dense references finish fast)
    "g_small": dict(N=6, m=(6, 12), mi=(1, 4), extra=4, l=2, li=1, n0=3, mi0=2, ng=2, me0=1,
                    f0=True, density=0.4),
    # medium: for the GPU
    "g_medium": dict(N=64, m=(48, 96), mi=(8, 24), extra=16, l=4, li=2, n0=8, mi0=4, ng=2,
                     me0=2, density=0.15),
    # large: 256 time blocks of 96..160 equality and 16..48 inequality rows
    "g_large": dict(N=256, m=(96, 160), mi=(16, 48), extra=32, l=8, li=4, n0=16, mi0=8, ng=4,
                    me0=2, density=0.10),
}


def generate_general(config="g_small", seed=0, **overrides) -> GeneralInstance:
    """Draw a feasible, bounded general instance.

    Draw order (PCG64(seed)): sizes (m_i, mi_i, then per block n_i = m_i + mi_i
    + extra), A_i, C_i, H_i, G_i per block, G_0, KR_j, KL_j per pair, the
    global rows' parts Wg_i (about 3 entries per row and block) and Wg_0, then
    per variable its bound kind and the interior point, then per inequality
    row its side kind and widths, then y, the inequality multipliers and the
    reduced costs.  Global rows 0, 2, ... are equalities, 1, 3, ...
    inequalities.  The x_0-only equality rows A_0 (drawn after the global
    rows, 60% dense, no zero rows) get b_0 = A_0 x_0 at the interior point;
    with f0, the equality link rows get an x_0 part F0 (50% dense), drawn
    after A_0.

    Bound kinds (probabilities): [0, inf) 0.4, [lo, up] 0.3, [lo, inf) 0.1,
    (-inf, up] 0.1, free 0.1.  The equality right-hand sides are the rows at
    an interior point xhat; inequality sides lie 0.1..1 from the row value at
    xhat (both sides 0.5, lower only 0.25, upper only 0.25).  The cost is
    c = Aeq'y + Ain'lam + r with lam and r signed as the dual of each bound
    and row kind requires (free variables r = 0), so the dual is feasible and
    the LP bounded.
    """
    cfg = dict(GENERAL_CONFIGS[config]) if isinstance(config, str) else dict(config)
    cfg.update(overrides)
    rng = np.random.Generator(np.random.PCG64(seed))
    N, n0, dens = int(cfg["N"]), int(cfg["n0"]), float(cfg["density"])

    def draw(spec, size):
        if isinstance(spec, tuple):
            return rng.integers(spec[0], spec[1] + 1, size=size).astype(np.int64)
        return np.full(size, spec, dtype=np.int64)

    m = draw(cfg["m"], N)
    mi = draw(cfg["mi"], N)
    n = m + mi + int(cfg["extra"])
    l = draw(cfg["l"], max(N - 1, 0))
    li = draw(cfg["li"], max(N - 1, 0))
    mi0 = int(cfg["mi0"])

    A, C, H, G = [], [], [], []
    for i in range(N):
        A.append(_sparse_block(rng, int(m[i]), int(n[i]), dens, True))
        C.append(_sparse_block(rng, int(m[i]), n0, dens, False))
        H.append(_sparse_block(rng, int(mi[i]), int(n[i]), dens, True))
        G.append(_sparse_block(rng, int(mi[i]), n0, dens, False))
    G0 = _sparse_block(rng, mi0, n0, max(dens, 0.5), True) if n0 > 0 else np.zeros((0, 0))
    if n0 == 0:
        mi0 = 0
    FR, FL, KR, KL = [], [], [], []
    for j in range(N - 1):
        lj, nj, nk = int(l[j]), int(n[j]), int(n[j + 1])
        fr = np.zeros((lj, nj)); fl = np.zeros((lj, nk))
        for k in range(lj):
            fr[k, nj - lj + k] = 1.0
            fl[k, k] = -1.0
        FR.append(fr); FL.append(fl)
        # inequality links on the next columns in from the boundary
        kr = np.zeros((int(li[j]), nj)); kl = np.zeros((int(li[j]), nk))
        for k in range(int(li[j])):
            kr[k, nj - lj - 1 - k] = rng.uniform(0.5, 1.5)
            kl[k, lj + k] = -rng.uniform(0.5, 1.5)
        KR.append(kr); KL.append(kl)
    # global rows: a few entries in every block (and on x_0); rows 0, 2, ...
    # are equalities, rows 1, 3, ... inequalities
    ng = int(cfg.get("ng", 0))
    Wg = [_sparse_block(rng, ng, int(n[i]), min(dens, 3.0 / float(n[i])), False) for i in range(N)]
    Wg0 = _sparse_block(rng, ng, n0, min(1.0, max(dens, 0.5)), False)
    geq = np.arange(ng) % 2 == 0
    me0 = int(cfg.get("me0", 0)) if n0 > 1 else 0
    A0 = _sparse_block(rng, me0, n0, 0.6, True) if me0 else None
    # equality link rows on x_0 (F0), where asked for
    F0 = _sparse_block(rng, int(l.sum()), n0, 0.5, False) if cfg.get("f0") and n0 else None

    nt = int(n.sum()) + n0
    kind = rng.choice(5, size=nt, p=[0.4, 0.3, 0.1, 0.1, 0.1])
    lo = np.zeros(nt); up = np.full(nt, np.inf); xhat = np.zeros(nt)
    a = rng.uniform(-1.0, 1.0, size=nt)
    w = rng.uniform(0.5, 3.0, size=nt)
    t = rng.uniform(0.2, 0.8, size=nt)
    for k in range(nt):
        if kind[k] == 0:
            lo[k], up[k], xhat[k] = 0.0, np.inf, 0.2 + 1.8 * t[k]
        elif kind[k] == 1:
            lo[k], up[k] = a[k], a[k] + w[k]
            xhat[k] = lo[k] + t[k] * w[k]
        elif kind[k] == 2:
            lo[k], up[k], xhat[k] = a[k], np.inf, a[k] + 0.2 + 1.8 * t[k]
        elif kind[k] == 3:
            lo[k], up[k], xhat[k] = -np.inf, a[k], a[k] - 0.2 - 1.8 * t[k]
        else:
            lo[k], up[k], xhat[k] = -np.inf, np.inf, a[k]

    inst = GeneralInstance(N=N, n0=n0, m=m, n=n, l=l, A=A, C=C, FR=FR, FL=FL, F0=F0,
                           b=np.zeros(int(m.sum() + l.sum())), H=H, G=G, d=[], f=[],
                           G0=G0, d0=np.zeros(mi0), f0=np.zeros(mi0), KR=KR, KL=KL, dl=[], fl=[],
                           c=np.zeros(nt), lo=lo, up=up, Wg=Wg, Wg0=Wg0,
                           dg=np.zeros(ng), fg=np.where(geq, 0.0, 1.0), A0=A0,
                           b0=np.zeros(me0), xhat=xhat)
    for i in range(N):
        inst.d.append(np.zeros(int(mi[i]))); inst.f.append(np.zeros(int(mi[i])))
    for j in range(N - 1):
        inst.dl.append(np.zeros(int(li[j]))); inst.fl.append(np.zeros(int(li[j])))
    Aeq, _, Ain, _, _ = general_matrices(inst)
    beq = Aeq @ xhat
    nb = int(m.sum() + l.sum())
    nge = int(geq.sum())
    inst.b = beq[:nb]
    inst.dg[geq] = beq[nb:nb + nge]
    inst.fg[geq] = beq[nb:nb + nge]
    inst.b0 = beq[nb + nge:]
    rhat = Ain @ xhat
    nin = rhat.size
    side = rng.choice(3, size=nin, p=[0.5, 0.25, 0.25])
    wd = rng.uniform(0.1, 1.0, size=nin)
    wf = rng.uniform(0.1, 1.0, size=nin)
    dv = np.where(side != 2, rhat - wd, -np.inf)
    fv = np.where(side != 1, rhat + wf, np.inf)
    # split the inequality sides back per group (same order as general_matrices)
    pos = 0
    for i in range(N):
        k = int(mi[i]); inst.d[i] = dv[pos:pos + k]; inst.f[i] = fv[pos:pos + k]; pos += k
    inst.d0 = dv[pos:pos + mi0]; inst.f0 = fv[pos:pos + mi0]; pos += mi0
    for j in range(N - 1):
        k = int(li[j]); inst.dl[j] = dv[pos:pos + k]; inst.fl[j] = fv[pos:pos + k]; pos += k
    inst.dg[~geq] = dv[pos:]
    inst.fg[~geq] = fv[pos:]
    # dual-feasible cost
    y = rng.standard_normal(Aeq.shape[0])
    lam_raw = rng.uniform(0.0, 1.0, size=nin)
    lam = np.where(side == 0, rng.standard_normal(nin), np.where(side == 1, lam_raw, -lam_raw))
    r_raw = rng.uniform(0.0, 1.0, size=nt)
    r = np.select([kind == 0, kind == 1, kind == 2, kind == 3],
                  [r_raw, rng.standard_normal(nt), r_raw, -r_raw], default=0.0)
    inst.c = Aeq.T @ y + Ain.T @ lam + r
    return inst
