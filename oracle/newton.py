"""Block-elimination Newton solve for the arrowhead LP (oracle).

Test infrastructure only (see package docstring).

What it computes.  The Newton system of Sec. 2.3 with dz eliminated is the
augmented system [[-(X^-1 Z), A'], [A, 0]] [dx; dy] = [rx - X^-1 rz; ry].
With primal regularization rho and dual regularization delta (a reading: the
paper leaves pivot handling to its sparse solvers) it becomes
[[-(X^-1 Z + rho I), A'], [A, delta I]].  Let D = (Z/X + rho)^-1.

Eliminating the block variables dx_i = D_i (A_i' dy_i + F_i' dy_L - rx^_i)
leaves an arrowhead system of the form of Sec. 3.2, eq. (compressed system),
with per-block normal matrices in place of the augmented blocks K_i:

    [ M_1             B_1 ] [dy_1 ]   M_i  = A_i D_i A_i' + delta I
    [      ...        ... ] [ ... ]   B_i  = [A_i D_i F_i' | C_i]
    [           M_N   B_N ] [dy_N ] = K0'  = [[sum F_i D_i F_i' + delta I, F0],
    [ B_1' ...  B_N'  K0' ] [dy_L ]           [F0',  -D_0^-1            ]]
                            [dx_0 ]

Factorization (Alg. 2): Cholesky of every M_i; the contributions B_i' M_i^-1 B_i
through W_i = L_i^-1 B_i; the sum S = K0' - sum_i W_i' W_i; the factorization
of S.  Because every link row touches two consecutive blocks only (Sec. 3.3),
S is block tridiagonal over the link pairs plus a dense border over x_0, as in
App. A, eq. (Schur block structure).  S is quasi-definite: its link part T is
positive definite and the border Schur complement negative definite, so S is
factored by two Choleskys: L_T (block bidiagonal, sequential over the pairs),
G = L_T^-1 E, and Lb = chol(-(S00 - G'G)).

Solve (Alg. 3): the Schur right-hand side b^_0 = b_0 - sum L_i' K_i^-1 b_i, the
Schur solve, the modified block right-hand sides and the block back-solves,
then dx and dz recovered by the elimination formulas.

Pivot rule (a reading; both implementations use it): inside a Cholesky a
pivot d <= 1e-30 * (max diagonal of the matrix handed to it) is replaced by
1e128 and counted.  For T the reference diagonal of pair j is the assembled
T_jj, so the threshold does not depend on the elimination order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.linalg as sla

from . import lp

# NumPy and SciPy each bundle an OpenBLAS with its own thread pool; two pools
# spinning on the same cores slow each other down tenfold.  The large products
# run through NumPy's pool, so SciPy's (small triangular solves, potrf) gets one
# thread.
try:
    from threadpoolctl import ThreadpoolController as _TC
    for _lib in _TC().lib_controllers:
        if "scipy.libs" in getattr(_lib, "filepath", "") and _lib.num_threads > 1:
            _lib.set_num_threads(1)
except Exception:  # pragma: no cover - threadpoolctl missing
    pass

PIVOT_REL = 1e-30
PIVOT_BIG = 1e128


def chol_rule(Mx, thr):
    """Lower Cholesky factor with the pivot rule; returns (L, replaced)."""
    k = Mx.shape[0]
    if k == 0:
        return np.zeros((0, 0)), 0
    c, info = sla.lapack.dpotrf(Mx, lower=1, clean=1)
    if info == 0 and np.all(np.diag(c) ** 2 > thr):
        return c, 0
    # Column-by-column Cholesky with the replacement rule.
    L = np.zeros_like(Mx)
    count = 0
    for j in range(k):
        d = Mx[j, j] - L[j, :j] @ L[j, :j]
        if not d > thr:
            d = PIVOT_BIG
            count += 1
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (Mx[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L, count


def _lsolve(L, B):
    if L.shape[0] == 0:
        return np.zeros_like(B)
    return sla.solve_triangular(L, B, lower=True, check_finite=False)


def _ltsolve(L, B):
    if L.shape[0] == 0:
        return np.zeros_like(B)
    return sla.solve_triangular(L, B, lower=True, trans="T", check_finite=False)


@dataclass
class Factor:
    inst: object
    x: np.ndarray
    z: np.ndarray
    D: np.ndarray
    rho: float
    delta: float
    L: List[np.ndarray] = field(default_factory=list)      # block Cholesky factors
    W: List[np.ndarray] = field(default_factory=list)      # L_i^-1 B_i
    Ld: List[np.ndarray] = field(default_factory=list)     # diagonal factors of T
    Ls: List[np.ndarray] = field(default_factory=list)     # L_T[j+1, j]
    G: np.ndarray = None                                   # L_T^-1 E
    Lb: np.ndarray = None                                  # chol(-(S00 - G'G))
    pivots: int = 0
    # assembled Schur complement (kept for structural tests)
    Td: List[np.ndarray] = field(default_factory=list)
    To: List[np.ndarray] = field(default_factory=list)     # T[j+1, j]
    E: np.ndarray = None
    S00: np.ndarray = None


def link_cols(inst, i):
    """(left, right) link matrices of block i: its part of pair i-1 and of
    pair i (empty matrices at the ends of the chain)."""
    ni = int(inst.n[i])
    left = inst.FL[i - 1] if i >= 1 else np.zeros((0, ni))
    right = inst.FR[i] if i <= inst.N - 2 else np.zeros((0, ni))
    return left, right


def schur_matrix_dense(f: Factor):
    """The assembled S as one dense array (tiny instances; structural tests)."""
    inst = f.inst
    lo = np.concatenate([[0], np.cumsum(inst.l)]).astype(np.int64)
    nl = int(lo[-1])
    S = np.zeros((nl + inst.n0, nl + inst.n0))
    for j in range(inst.N - 1):
        S[lo[j]:lo[j + 1], lo[j]:lo[j + 1]] = f.Td[j]
        if j + 1 < inst.N - 1:
            S[lo[j + 1]:lo[j + 2], lo[j]:lo[j + 1]] = f.To[j]
            S[lo[j]:lo[j + 1], lo[j + 1]:lo[j + 2]] = f.To[j].T
    S[:nl, nl:] = f.E
    S[nl:, :nl] = f.E.T
    S[nl:, nl:] = f.S00
    return S


def factor(inst, x, z, rho=0.0, delta=0.0):
    """Alg. 2 for the normal-equation arrowhead form above."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(z))):
        raise FloatingPointError("non-finite x or z")
    if np.any(x <= 0) or np.any(z <= 0):
        raise FloatingPointError("x and z must be positive")
    D = 1.0 / (z / x + rho)
    xo, yo, lo = lp.offsets(inst)
    N, n0 = inst.N, inst.n0
    f = Factor(inst=inst, x=x, z=z, D=D, rho=rho, delta=delta)
    P = N - 1

    # Schur complement starts from K0' (Alg. 2 step 3 sums into it)
    Td = [delta * np.eye(int(inst.l[j])) for j in range(P)]
    To = [np.zeros((int(inst.l[j + 1]), int(inst.l[j]))) for j in range(P - 1)]
    E = np.zeros((int(lo[-1]), n0)) if inst.F0 is None else inst.F0.copy()
    S00 = -np.diag(1.0 / D[xo[-1]:])

    for i in range(N):   # Alg. 2 steps 1-2 for every block (increasing i)
        Ai = inst.A[i]
        Di = D[xo[i]:xo[i + 1]]
        Mi = (Ai * Di) @ Ai.T + delta * np.eye(Ai.shape[0])
        Li, cnt = chol_rule(Mi, PIVOT_REL * max(float(np.max(np.diag(Mi), initial=0.0)), 0.0))
        f.pivots += cnt
        left, right = link_cols(inst, i)
        Bi = np.hstack([(Ai * Di) @ left.T, (Ai * Di) @ right.T, inst.C[i]])
        Wi = _lsolve(Li, Bi)
        f.L.append(Li)
        f.W.append(Wi)
        # step 3: add K0' pieces of this block and subtract W_i' W_i
        Q = Wi.T @ Wi
        nl_, nr_ = left.shape[0], right.shape[0]
        FDF_ll = (left * Di) @ left.T
        FDF_rr = (right * Di) @ right.T
        FDF_rl = (right * Di) @ left.T
        sl = slice(0, nl_)
        sr = slice(nl_, nl_ + nr_)
        s0 = slice(nl_ + nr_, nl_ + nr_ + n0)
        if i >= 1:      # pair i-1 (left)
            Td[i - 1] += FDF_ll - Q[sl, sl]
            E[lo[i - 1]:lo[i]] -= Q[sl, s0]
        if i <= N - 2:  # pair i (right)
            Td[i] += FDF_rr - Q[sr, sr]
            E[lo[i]:lo[i + 1]] -= Q[sr, s0]
        if 1 <= i <= N - 2:  # coupling of pair i with pair i-1
            To[i - 1] += FDF_rl - Q[sr, sl]
        S00 -= Q[s0, s0]
    f.Td, f.To, f.E, f.S00 = Td, To, E, S00

    # Alg. 2 step 4: factor S (block-tridiagonal Cholesky, then the border)
    for j in range(P):
        X = Td[j].copy()
        if j > 0:
            X -= f.Ls[j - 1] @ f.Ls[j - 1].T
        thr = PIVOT_REL * max(float(np.max(np.diag(Td[j]), initial=0.0)), 0.0)
        Lj, cnt = chol_rule(X, thr)
        f.pivots += cnt
        f.Ld.append(Lj)
        if j < P - 1:
            f.Ls.append(_lsolve(Lj, To[j].T).T)           # To[j] Lj^-T
    G = np.zeros_like(E)
    for j in range(P):
        rhs = E[lo[j]:lo[j + 1]].copy()
        if j > 0:
            rhs -= f.Ls[j - 1] @ G[lo[j - 1]:lo[j]]
        G[lo[j]:lo[j + 1]] = _lsolve(f.Ld[j], rhs)
    f.G = G
    B = -(S00 - G.T @ G)
    Lb, cnt = chol_rule(B, PIVOT_REL * max(float(np.max(np.diag(B), initial=0.0)), 0.0))
    f.pivots += cnt
    f.Lb = Lb
    return f


def schur_solve(f: Factor, sL, s0):
    """Solve S [uL; u0] = [sL; s0] with the quasi-definite factorization."""
    inst = f.inst
    lo = np.concatenate([[0], np.cumsum(inst.l)]).astype(np.int64)
    P = inst.N - 1
    w = np.zeros_like(sL)
    for j in range(P):
        r = sL[lo[j]:lo[j + 1]].copy()
        if j > 0:
            r -= f.Ls[j - 1] @ w[lo[j - 1]:lo[j]]
        w[lo[j]:lo[j + 1]] = _lsolve(f.Ld[j], r)
    t = s0 - f.G.T @ w
    u0 = -_ltsolve(f.Lb, _lsolve(f.Lb, t))
    w = w - f.G @ u0
    uL = np.zeros_like(sL)
    for j in reversed(range(P)):
        r = w[lo[j]:lo[j + 1]].copy()
        if j < P - 1:
            r -= f.Ls[j].T @ uL[lo[j + 1]:lo[j + 2]]
        uL[lo[j]:lo[j + 1]] = _ltsolve(f.Ld[j], r)
    return uL, u0


def solve(f: Factor, rx, ry, rz):
    """Alg. 3: returns (dx, dy, dz) for the right-hand side (rx, ry, rz)."""
    inst = f.inst
    xo, yo, lo = lp.offsets(inst)
    N, n0 = inst.N, inst.n0
    rhx = rx - rz / f.x
    D = f.D
    sL = ry[yo[-1]:].copy()
    s0 = rhx[xo[-1]:].copy()
    V = []
    for i in range(N):     # Alg. 3 steps 1-2
        Di = D[xo[i]:xo[i + 1]]
        ri = rhx[xo[i]:xo[i + 1]]
        t = ry[yo[i]:yo[i + 1]] + inst.A[i] @ (Di * ri)
        v = _lsolve(f.L[i], t)
        V.append(v)
        q = f.W[i].T @ v
        left, right = link_cols(inst, i)
        nl_, nr_ = left.shape[0], right.shape[0]
        if i >= 1:
            sL[lo[i - 1]:lo[i]] += left @ (Di * ri) - q[:nl_]
        if i <= N - 2:
            sL[lo[i]:lo[i + 1]] += right @ (Di * ri) - q[nl_:nl_ + nr_]
        s0 -= q[nl_ + nr_:]
    uL, u0 = schur_solve(f, sL, s0)   # step 3
    dx = np.empty(int(xo[-1]) + n0)
    dy = np.empty(int(yo[-1] + lo[-1]))
    for i in range(N):     # steps 4-5, then dx by the elimination formula
        left, right = link_cols(inst, i)
        ul = uL[lo[i - 1]:lo[i]] if i >= 1 else np.zeros(0)
        ur = uL[lo[i]:lo[i + 1]] if i <= N - 2 else np.zeros(0)
        ui = np.concatenate([ul, ur, u0])
        dyi = _ltsolve(f.L[i], V[i] - f.W[i] @ ui)
        dy[yo[i]:yo[i + 1]] = dyi
        Di = D[xo[i]:xo[i + 1]]
        g = inst.A[i].T @ dyi + left.T @ ul + right.T @ ur
        dx[xo[i]:xo[i + 1]] = Di * (g - rhx[xo[i]:xo[i + 1]])
    dy[yo[-1]:] = uL
    dx[xo[-1]:] = u0
    dz = (rz - f.z * dx) / f.x
    return dx, dy, dz
