"""Seeded synthetic arrowhead LPs with a known optimum.

This module only draws problem data; it contains none of the interior-point
method's arithmetic, so both the GPU path and the CPU oracle may use it.

The LP is the standard-form problem of Sec. 2.2 (min c'x, Ax = b, x >= 0) with
the arrowhead block structure of Sec. 3.2, restricted to equality rows,
x >= 0 bounds and local (two-link) linking constraints (Sec. 3.3):

    block rows   A_i x_i + C_i x_0                   = b_i      i = 1..N
    link rows    FR_j x_j + FL_j x_{j+1} + F0_j x_0  = b_Lj     j = 1..N-1

Here ``A_i`` is the paper's B_i, ``C_i`` the paper's A_i (coupling to the
linking variables x_0), ``FR_j`` the paper's local block F_j and ``FL_j`` the
paper's F'_j.  Canonical vector order: x = [x_1..x_N, x_0], y = [y_1..y_N, y_L]
with y_L listing the link pairs in order.

Known optimum (complementary primal/dual pair chosen first, data derived):
  * x*: in every block exactly floor(n_i/2) entries ~U[0.5, 2], the rest 0;
    the same for x_0 with floor(n0/2);
  * z*: ~U[0.5, 2] where x* = 0, else 0;  y* ~ N(0, 1);
  * b = A x*,  c = A' y* + z*,  so f* = c'x* = b'y*.

Storage-continuity links: row k of pair j has +1 on variable n_j - l_j + k of
block j and -1 on variable k of block j+1 (energy-system storage balance).

Draw order (fixed; PCG64(seed)): random sizes (m_i, then l_j), then per block
A_i (mask, values, zero-row redraws) and C_i (mask, values), then x* positions
and values per block and for x_0, then z* values, then y*.

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
    b: np.ndarray
    c: np.ndarray
    xstar: np.ndarray = field(default=None)
    ystar: np.ndarray = field(default=None)
    zstar: np.ndarray = field(default=None)
    fstar: float = float("nan")
    basis: Optional[list] = field(default=None)   # nondegenerate variant: positive x* indices per block

    @property
    def n_tot(self) -> int:
        return int(self.n.sum()) + self.n0

    @property
    def m_tot(self) -> int:
        return int(self.m.sum()) + int(self.l.sum())

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
    m_tot = int(m.sum() + l.sum())
    ystar = rng.standard_normal(m_tot)

    inst = Instance(N=N, n0=n0, m=m, n=n, l=l, A=A, C=C, FR=FR, FL=FL, F0=F0,
                    b=np.zeros(m_tot), c=np.zeros(xstar.size))
    inst.xstar, inst.ystar, inst.zstar = xstar, ystar, zstar
    inst.basis = basis   # per block: the indices of the positive x* entries (nondegenerate only)
    inst.b = apply_A(inst, xstar)
    inst.c = apply_At(inst, ystar) + zstar
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
    return out
