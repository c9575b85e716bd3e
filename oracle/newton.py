"""Block-elimination Newton solve for the arrowhead LP (oracle).

Test infrastructure only (see package docstring).

What it computes.  The Newton system of Sec. 2.3 with dz eliminated is the
augmented system [[-(X^-1 Z), A'], [A, 0]] [dx; dy] = [rx - X^-1 rz; ry].
With primal regularization rho and dual regularization delta (a reading: the
paper leaves pivot handling to its sparse solvers) it becomes
[[-(X^-1 Z + rho I), A'], [A, delta I]].  Let D = (Z/X + rho)^-1.

Eliminating the block variables dx_i = D_i (A_i' dy_i + F_i' dy_L + Wg_i' dy_G
- rx^_i) leaves an arrowhead system of the form of Sec. 3.2, eq. (compressed
system), with per-block normal matrices in place of the augmented blocks K_i
(F_i: block i's part of the link rows, Wg_i: of the global rows):

    [ M_1             B_1 ] [dy_1 ]   M_i  = A_i D_i A_i' + delta I
    [      ...        ... ] [ ... ]   B_i  = [A_i D_i F_i' | A_i D_i Wg_i' | C_i]
    [           M_N   B_N ] [dy_N ] = K0'  = [[FDF' + dI, FDWg',      F0 ],
    [ B_1' ...  B_N'  K0' ] [dy_L ]           [WgDF',    WgDWg' + dI, Wg0],
                            [dy_G ]           [F0',      Wg0',  -D_0^-1  ]]
                            [dx_0 ]
(sums over the blocks).

Factorization (Alg. 2): Cholesky of every M_i; the contributions B_i' M_i^-1 B_i
through W_i = L_i^-1 B_i; the sum S = K0' - sum_i W_i' W_i; the factorization
of S.  Because every link row touches two consecutive blocks only (Sec. 3.3),
S is block tridiagonal over the link pairs plus a dense border over the global
rows and x_0 (the dense layer of Sec. 4.1; App. A, eq. (Schur block structure),
for the local part).  S is quasi-definite: its dual part (link and global rows)
is positive definite and its x_0 part negative definite.  It is factored by
Choleskys: L_T (block bidiagonal, sequential over the pairs), G = L_T^-1 E,
then the border Schur complement Sb = S00 - G'G (global rows first, then x_0):
Lg = chol(Sb_gg), X = Lg^-1 Sb_g0, Lx = chol(-(Sb_00 - X'X)), so that
Sb = Lb diag(I, -I) Lb' with Lb = [[Lg, 0], [X', Lx]].  Without global rows
this is Lb = chol(-(S00 - G'G)).

Solve (Alg. 3): the Schur right-hand side b^_0 = b_0 - sum L_i' K_i^-1 b_i, the
Schur solve, the modified block right-hand sides and the block back-solves,
then dx and dz recovered by the elimination formulas.

Pivot rule (a reading; both implementations use it): inside a Cholesky a
pivot d <= 1e-30 * (max diagonal of the matrix handed to it) is replaced by
1e128 and counted.  For T the reference diagonal of pair j is the assembled
T_jj, so the threshold does not depend on the elimination order.  Both
Choleskys of the border take 1e-30 * the largest |diagonal entry| of Sb.
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
    Lb: np.ndarray = None                                  # border factor, Sb = Lb diag(I, -I) Lb'
    ng: int = 0                                            # global rows (the + part of the border)
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


def global_cols(inst, i):
    """Block i's part of the global rows (ng x n_i; 0 x n_i without any)."""
    if lp.ng(inst) == 0:
        return np.zeros((0, int(inst.n[i])))
    return inst.Wg[i]


def schur_matrix_dense(f: Factor):
    """The assembled S as one dense array over (y_L, y_G, x_0) (tiny
    instances; structural tests)."""
    inst = f.inst
    lo = np.concatenate([[0], np.cumsum(inst.l)]).astype(np.int64)
    nl = int(lo[-1])
    nb = f.ng + inst.n0
    S = np.zeros((nl + nb, nl + nb))
    for j in range(inst.N - 1):
        S[lo[j]:lo[j + 1], lo[j]:lo[j + 1]] = f.Td[j]
        if j + 1 < inst.N - 1:
            S[lo[j + 1]:lo[j + 2], lo[j]:lo[j + 1]] = f.To[j]
            S[lo[j]:lo[j + 1], lo[j + 1]:lo[j + 2]] = f.To[j].T
    S[:nl, nl:] = f.E
    S[nl:, :nl] = f.E.T
    S[nl:, nl:] = f.S00
    return S


def factor(inst, x, z, rho=0.0, delta=0.0, q=None):
    """Alg. 2 for the normal-equation arrowhead form above.  q (>= 0, one per
    variable): an extra diagonal of the (x, x) block, -(X^-1 Z + Q + rho I),
    which is where upper bounds handled inside the iteration enter (q = w / s,
    0 for a variable without one); D = (Z/X + q + rho)^-1."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(z))):
        raise FloatingPointError("non-finite x or z")
    if np.any(x <= 0) or np.any(z <= 0):
        raise FloatingPointError("x and z must be positive")
    D = 1.0 / (z / x + rho) if q is None else 1.0 / (z / x + q + rho)
    xo, yo, lo = lp.offsets(inst)
    N, n0, ng = inst.N, inst.n0, lp.ng(inst)
    f = Factor(inst=inst, x=x, z=z, D=D, rho=rho, delta=delta, ng=ng)
    P = N - 1

    # Schur complement starts from K0' (Alg. 2 step 3 sums into it); the
    # border columns are the global rows, then x_0
    Td = [delta * np.eye(int(inst.l[j])) for j in range(P)]
    To = [np.zeros((int(inst.l[j + 1]), int(inst.l[j]))) for j in range(P - 1)]
    E = np.zeros((int(lo[-1]), ng + n0))
    if inst.F0 is not None:
        E[:, ng:] = inst.F0
    S00 = np.zeros((ng + n0, ng + n0))
    S00[:ng, :ng] = delta * np.eye(ng)
    if ng:
        S00[:ng, ng:] = inst.Wg0
        S00[ng:, :ng] = inst.Wg0.T
    S00[ng:, ng:] = -np.diag(1.0 / D[xo[-1]:])

    for i in range(N):   # Alg. 2 steps 1-2 for every block (increasing i)
        Ai = inst.A[i]
        Di = D[xo[i]:xo[i + 1]]
        Mi = (Ai * Di) @ Ai.T + delta * np.eye(Ai.shape[0])
        Li, cnt = chol_rule(Mi, PIVOT_REL * max(float(np.max(np.diag(Mi), initial=0.0)), 0.0))
        f.pivots += cnt
        left, right = link_cols(inst, i)
        glob = global_cols(inst, i)
        Bi = np.hstack([(Ai * Di) @ left.T, (Ai * Di) @ right.T, (Ai * Di) @ glob.T, inst.C[i]])
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
        sb = slice(nl_ + nr_, nl_ + nr_ + ng + n0)    # border: global rows, then x_0
        FDB_l = np.hstack([(left * Di) @ glob.T, np.zeros((nl_, n0))])
        FDB_r = np.hstack([(right * Di) @ glob.T, np.zeros((nr_, n0))])
        BDB = np.zeros((ng + n0, ng + n0))
        BDB[:ng, :ng] = (glob * Di) @ glob.T
        if i >= 1:      # pair i-1 (left)
            Td[i - 1] += FDF_ll - Q[sl, sl]
            E[lo[i - 1]:lo[i]] += FDB_l - Q[sl, sb]
        if i <= N - 2:  # pair i (right)
            Td[i] += FDF_rr - Q[sr, sr]
            E[lo[i]:lo[i + 1]] += FDB_r - Q[sr, sb]
        if 1 <= i <= N - 2:  # coupling of pair i with pair i-1
            To[i - 1] += FDF_rl - Q[sr, sl]
        S00 += BDB - Q[sb, sb]
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
    # border (dense layer): Sb = S00 - G'G is quasi-definite, + on the global
    # rows and - on x_0
    Sb = S00 - G.T @ G
    thr = PIVOT_REL * float(np.max(np.abs(np.diag(Sb)), initial=0.0))
    Lg, cnt = chol_rule(Sb[:ng, :ng], thr)
    f.pivots += cnt
    X = _lsolve(Lg, Sb[:ng, ng:])
    Lx, cnt = chol_rule(-(Sb[ng:, ng:] - X.T @ X), thr)
    f.pivots += cnt
    Lb = np.zeros_like(Sb)
    Lb[:ng, :ng] = Lg
    Lb[ng:, :ng] = X.T
    Lb[ng:, ng:] = Lx
    f.Lb = Lb
    return f


def border_solve(f: Factor, t):
    """u with Sb u = t, from Sb = Lb diag(I_ng, -I_n0) Lb'."""
    w = _lsolve(f.Lb, t)
    w[f.ng:] = -w[f.ng:]
    return _ltsolve(f.Lb, w)


def schur_solve(f: Factor, sL, s0):
    """Solve S [uL; u0] = [sL; s0] with the quasi-definite factorization; the
    border parts s0, u0 hold the global rows, then x_0."""
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
    u0 = border_solve(f, t)
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
    N, n0, ng = inst.N, inst.n0, f.ng
    nl = int(lo[-1])
    rhx = rx - rz / f.x
    D = f.D
    sL = ry[yo[-1]:yo[-1] + nl].copy()
    s0 = np.concatenate([ry[yo[-1] + nl:], rhx[xo[-1]:]])   # global rows, then x_0
    V = []
    for i in range(N):     # Alg. 3 steps 1-2
        Di = D[xo[i]:xo[i + 1]]
        ri = rhx[xo[i]:xo[i + 1]]
        t = ry[yo[i]:yo[i + 1]] + inst.A[i] @ (Di * ri)
        v = _lsolve(f.L[i], t)
        V.append(v)
        q = f.W[i].T @ v
        left, right = link_cols(inst, i)
        glob = global_cols(inst, i)
        nl_, nr_ = left.shape[0], right.shape[0]
        if i >= 1:
            sL[lo[i - 1]:lo[i]] += left @ (Di * ri) - q[:nl_]
        if i <= N - 2:
            sL[lo[i]:lo[i + 1]] += right @ (Di * ri) - q[nl_:nl_ + nr_]
        s0[:ng] += glob @ (Di * ri)
        s0 -= q[nl_ + nr_:]
    uL, u0 = schur_solve(f, sL, s0)   # step 3
    dx = np.empty(int(xo[-1]) + n0)
    dy = np.empty(int(yo[-1]) + nl + ng)
    for i in range(N):     # steps 4-5, then dx by the elimination formula
        left, right = link_cols(inst, i)
        glob = global_cols(inst, i)
        ul = uL[lo[i - 1]:lo[i]] if i >= 1 else np.zeros(0)
        ur = uL[lo[i]:lo[i + 1]] if i <= N - 2 else np.zeros(0)
        ui = np.concatenate([ul, ur, u0])
        dyi = _ltsolve(f.L[i], V[i] - f.W[i] @ ui)
        dy[yo[i]:yo[i + 1]] = dyi
        Di = D[xo[i]:xo[i + 1]]
        g = inst.A[i].T @ dyi + left.T @ ul + right.T @ ur + glob.T @ u0[:ng]
        dx[xo[i]:xo[i + 1]] = Di * (g - rhx[xo[i]:xo[i + 1]])
    dy[yo[-1]:yo[-1] + nl] = uL
    dy[yo[-1] + nl:] = u0[:ng]
    dx[xo[-1]:] = u0[ng:]
    dz = (rz - f.z * dx) / f.x
    return dx, dy, dz
