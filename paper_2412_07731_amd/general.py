"""General arrowhead LPs (inequality rows and variable bounds, the form of
Sec. 3.2) solved through the standard-form library.

The conversion is exact and keeps the arrowhead structure, so every
interior-point iteration still runs in libahlp's kernels:

  * a variable with a finite lower bound is shifted, x = lo + x' (x' >= 0);
    one with only an upper bound is flipped, x = up - x'; a free one is
    split, x = x+ - x-;
  * an inequality row d <= r(x) <= f becomes r(x) - t = 0 with a slack t of
    bounds [d, f] placed in the row's block (the left block for a link pair,
    the first block for x_0-only rows), converted like a variable;
  * every remaining finite upper bound u' gets a slack row x' + s = u' in the
    variable's block (the first block for x_0);
  * a global row dg <= sum_i Wg_i x_i + Wg_0 x_0 <= fg is chained through the
    blocks: block i gets the partial sum s_i = s_{i-1} + Wg_i x_i as a new
    free variable (block 1's includes Wg_0 x_0), block 1 a row defining s_1,
    link pair i a row s_{i+1} - s_i - Wg_{i+1} x_{i+1} = 0, and the last
    partial sum takes the row's sides as bounds.  An equality row has no last
    partial sum: its last link row (its block row when N = 1) carries the
    right-hand side.  Global rows thus become local two-links (done first,
    by chain_globals);
  * equality rows on x_0 alone, A_0 x_0 = b_0 (full row rank), are solved for
    r = rank basic entries of x_0 chosen by a column-pivoted QR of A_0:
    x_B = B^-1 (b_0 - A_0,N x_N).  x_N stay the linking variables with their
    bounds, x_B is substituted in every row, and x_B's bounds become x_0-only
    inequality rows on x_N (done before everything else, by eliminate_x0_rows).

Layout after chain_globals: block i's variables are its own, then its partial
sums s_{k,i} for k = 0, 1, ... (where they exist); block 1's equality rows are
its own, then one per global row; link pair j's equality rows are its own,
then one per global row.

Standard-form layout of block i (columns):
  1. its n_i variables (x', or x+ of a free variable), in order;
  2. x- of its free variables, in order;
  3. t' of its inequality rows, then of the inequality rows of link pair i
     (pair i joins blocks i and i+1), then (first block only) of the x_0-only
     inequality rows;
  4. the upper-bound slacks s of the columns of 1-3 with a finite bound, in
     column order, then (first block only) those of the x_0 columns.
Rows of block i: its equality rows, its inequality rows (then, first block,
the x_0-only ones), then the upper-bound rows in the order of 4.  x_0: its
n0 columns, then x- of its free entries.  Link pair j: its equality rows,
then its inequality rows.

Dense layer (to_standard(g, dense=True)): the global rows stay whole, as
global rows of the standard form, which the library keeps in the border of
the Schur complement (the dense layer of Sec. 4.1) instead of chaining them
through the blocks.  The x_0-only equality rows are still eliminated, unless
x0_border=True keeps them whole as global rows too (with no block part; the
border then carries rows whose diagonal is only the regularization delta,
which costs refinement corrections).  An inequality global
row dg <= r(x) <= fg becomes r(x) - t = 0 with its slack t a new linking
variable: x_0's columns are its own, x- of its free entries, then these
slacks in global row order (their upper-bound slacks, when both sides are
finite, join block 1's like those of the other x_0 columns).  Global rows of
the standard form: those of g in order, then the x_0-only equality rows.

Bounds inside the iteration (to_standard(g, bounds=True)): the finite upper
bounds left after the shifts stay bounds of the standard columns (Instance.ub)
instead of becoming rows x' + s = u' (step 4 of the layout is skipped), and
the library's interior-point method handles them with slacks and duals of its
own.

Only the primal solution is mapped back; duals of the general form are not.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .gen import GeneralInstance, Instance


@dataclass
class StandardMap:
    """x = off + T x_std for each block (and x_0); objective constant; keep:
    the original variables among those of the chained form (None: all)."""
    T: List[np.ndarray]        # per block: n_i x ncol_i, then x_0: n0 x n0_std
    off: List[np.ndarray]
    xoff_std: np.ndarray       # block starts in the standard x (length N+1)
    const: float
    keep: np.ndarray = None
    x0map: tuple = None        # (e, E, x_0 start): x_0 = e + E x_N


def _var_map(lo, up):
    """Per variable: (column sign matrix part, offset, upper bound after the
    shift or inf, is_free).  Returns T0 (k x (k + nfree)), off, ubound of the
    k primary columns, and the list of free indices."""
    k = lo.size
    free = [v for v in range(k) if not np.isfinite(lo[v]) and not np.isfinite(up[v])]
    T = np.zeros((k, k + len(free)))
    off = np.zeros(k)
    ub = np.full(k, np.inf)
    for v in range(k):
        if np.isfinite(lo[v]):
            T[v, v] = 1.0
            off[v] = lo[v]
            ub[v] = up[v] - lo[v]
        elif np.isfinite(up[v]):
            T[v, v] = -1.0
            off[v] = up[v]
        else:
            T[v, v] = 1.0
    for q, v in enumerate(free):
        T[v, k + q] = -1.0
    return T, off, ub


def _slack_col(dv, fv):
    """Slack t of a row with sides [d, f]: (sign of t' in t, offset, upper bound of t')."""
    if np.isfinite(dv):
        return 1.0, dv, (fv - dv) if np.isfinite(fv) else np.inf
    return -1.0, fv, np.inf


def eliminate_x0_rows(g: GeneralInstance):
    """The same LP without x_0-only equality rows: x_0 = e + E x_N.  Returns
    the reduced instance, e and E."""
    import copy
    import scipy.linalg as sla
    me0 = 0 if g.A0 is None else g.A0.shape[0]
    n0 = g.n0
    if me0 == 0:
        return g, np.zeros(n0), np.eye(n0)
    _, _, perm = sla.qr(g.A0, pivoting=True)
    bas, non = perm[:me0], perm[me0:]
    Binv = np.linalg.inv(g.A0[:, bas])
    pB = Binv @ g.b0
    QB = -Binv @ g.A0[:, non]
    E = np.zeros((n0, non.size))
    e = np.zeros(n0)
    E[non, np.arange(non.size)] = 1.0
    E[bas] = QB
    e[bas] = pB
    h = copy.copy(g)
    xo0 = int(g.n.sum())
    h.n0 = int(non.size)
    h.C = [Ci @ E for Ci in g.C]
    h.G = [Gi @ E for Gi in g.G]
    h.b = g.b.copy()
    mb = int(g.m.sum())
    for i in range(g.N):
        h.b[int(g.m[:i].sum()):int(g.m[:i + 1].sum())] -= g.C[i] @ e
    h.d = [g.d[i] - g.G[i] @ e for i in range(g.N)]
    h.f = [g.f[i] - g.G[i] @ e for i in range(g.N)]
    if g.F0 is not None:
        h.F0 = g.F0 @ E
        h.b[mb:] -= g.F0 @ e
    if g.ng:
        h.Wg0 = g.Wg0 @ E
        h.dg = g.dg - g.Wg0 @ e
        h.fg = g.fg - g.Wg0 @ e
    # x_0-only inequality rows: the existing ones, then the bounds of x_B
    lo0, up0 = g.lo[xo0:], g.up[xo0:]
    rows = [g.G0 @ E] if g.G0.size else []
    dd = [g.d0 - g.G0 @ e] if g.G0.size else []
    ff = [g.f0 - g.G0 @ e] if g.G0.size else []
    for q, j in enumerate(bas):
        if np.isfinite(lo0[j]) or np.isfinite(up0[j]):
            rows.append(QB[q:q + 1])
            dd.append(np.array([lo0[j] - pB[q]]))
            ff.append(np.array([up0[j] - pB[q]]))
    h.G0 = np.vstack(rows) if rows else np.zeros((0, h.n0))
    h.d0 = np.concatenate(dd) if dd else np.zeros(0)
    h.f0 = np.concatenate(ff) if ff else np.zeros(0)
    h.c = np.concatenate([g.c[:xo0], E.T @ g.c[xo0:]])
    h.lo = np.concatenate([g.lo[:xo0], lo0[non]])
    h.up = np.concatenate([g.up[:xo0], up0[non]])
    h.A0 = None
    h.b0 = np.zeros(0)
    return h, e, E


def chain_globals(g: GeneralInstance) -> GeneralInstance:
    """The same LP with every global row replaced by a chain of partial sums
    (local two-links); the original variables stay first in each block."""
    if g.ng == 0:
        return g
    N, n0, ng = g.N, g.n0, g.ng
    is_eq = g.dg == g.fg
    # which partial sums exist: s_{k,i} for i < N-1, and the last for inequalities
    has = np.ones((ng, N), dtype=bool)
    has[is_eq, N - 1] = False
    nsum = has.sum(axis=0)                          # new variables per block
    col = np.cumsum(has, axis=0) - 1                # index of s_{k,i} among block i's sums
    xo = np.concatenate([[0], np.cumsum(g.n)]).astype(np.int64)
    n_new = g.n + nsum
    lo, up, c = [], [], []
    for i in range(N):
        sl = slice(xo[i], xo[i + 1])
        lo_s = np.full(int(nsum[i]), -np.inf)
        up_s = np.full(int(nsum[i]), np.inf)
        if i == N - 1:
            for k in range(ng):
                if has[k, i]:
                    lo_s[col[k, i]] = g.dg[k]
                    up_s[col[k, i]] = g.fg[k]
        lo += [g.lo[sl], lo_s]
        up += [g.up[sl], up_s]
        c += [g.c[sl], np.zeros(int(nsum[i]))]
    lo += [g.lo[xo[-1]:]]
    up += [g.up[xo[-1]:]]
    c += [g.c[xo[-1]:]]
    pad = lambda X, i: np.hstack([X, np.zeros((X.shape[0], int(nsum[i])))])
    A = [pad(g.A[i], i) for i in range(N)]
    C = [g.C[i].copy() for i in range(N)]
    H = [pad(g.H[i], i) for i in range(N)]
    KR = [pad(g.KR[j], j) for j in range(N - 1)]
    KL = [pad(g.KL[j], j + 1) for j in range(N - 1)]
    FR = [pad(g.FR[j], j) for j in range(N - 1)]
    FL = [pad(g.FL[j], j + 1) for j in range(N - 1)]
    mb = int(g.m.sum())
    bb = [g.b[int(g.m[:i].sum()):int(g.m[:i + 1].sum())] for i in range(N)]
    lofs = np.concatenate([[0], np.cumsum(g.l)]).astype(np.int64)
    bl = [g.b[mb + lofs[j]: mb + lofs[j + 1]] for j in range(N - 1)]
    F0 = [g.F0[lofs[j]:lofs[j + 1]] if g.F0 is not None else np.zeros((int(g.l[j]), n0))
          for j in range(N - 1)]
    # block 1: s_{k,0} - Wg_0 x_1 - Wg0 x_0 = 0 (or, with no s_{k,0}, the row itself)
    R = np.zeros((ng, int(n_new[0])))
    R[:, :int(g.n[0])] = -g.Wg[0]
    RC = -g.Wg0 if n0 else np.zeros((ng, 0))
    rb = np.zeros(ng)
    for k in range(ng):
        if has[k, 0]:
            R[k, int(g.n[0]) + col[k, 0]] = 1.0
        else:
            rb[k] = -g.dg[k]
    A[0] = np.vstack([A[0], R])
    C[0] = np.vstack([C[0], RC])
    bb[0] = np.concatenate([bb[0], rb])
    # pair j: s_{k,j+1} - s_{k,j} - Wg_{j+1} x_{j+1} = 0 (or = -dg at the end of an equality)
    for j in range(N - 1):
        fr = np.zeros((ng, int(n_new[j])))
        fl = np.zeros((ng, int(n_new[j + 1])))
        fl[:, :int(g.n[j + 1])] = -g.Wg[j + 1]
        rj = np.zeros(ng)
        for k in range(ng):
            fr[k, int(g.n[j]) + col[k, j]] = -1.0
            if has[k, j + 1]:
                fl[k, int(g.n[j + 1]) + col[k, j + 1]] = 1.0
            else:
                rj[k] = -g.dg[k]
        FR[j] = np.vstack([FR[j], fr])
        FL[j] = np.vstack([FL[j], fl])
        F0[j] = np.vstack([F0[j], np.zeros((ng, n0))])
        bl[j] = np.concatenate([bl[j], rj])
    F0all = np.vstack(F0) if F0 and (g.F0 is not None) else None
    out = GeneralInstance(
        N=N, n0=n0, m=g.m + np.eye(N, dtype=np.int64)[0] * ng, n=n_new, l=g.l + ng, A=A, C=C,
        FR=FR, FL=FL, F0=F0all, b=np.concatenate(bb + bl), H=H, G=[x.copy() for x in g.G],
        d=g.d, f=g.f, G0=g.G0, d0=g.d0, f0=g.f0, KR=KR, KL=KL, dl=g.dl, fl=g.fl,
        c=np.concatenate(c), lo=np.concatenate(lo), up=np.concatenate(up))
    out.orig_cols = np.concatenate([np.arange(xo[i] + np.sum(nsum[:i]), xo[i + 1] + np.sum(nsum[:i]))
                                    for i in range(N)]
                                   + [np.arange(int(n_new.sum()), int(n_new.sum()) + n0)])
    return out


def to_standard(g: GeneralInstance, dense=False, x0_border=False, bounds=False):
    """The equivalent standard-form Instance and the map back to x (global
    rows chained, x_0-only equality rows eliminated; with dense, the global
    rows kept whole as global rows, and with x0_border the x_0-only rows
    too)."""
    if not (dense and x0_border) and g.A0 is not None and g.A0.shape[0]:
        h, e, E = eliminate_x0_rows(g)
        inst, mp = to_standard(h, dense=dense, bounds=bounds)
        mp.x0map = (e, E, int(g.n.sum()))
        return inst, mp
    if not dense and g.ng:
        gc = chain_globals(g)
        inst, mp = to_standard(gc, bounds=bounds)
        mp.keep = gc.orig_cols
        return inst, mp
    N, n0 = g.N, g.n0
    xo = np.concatenate([[0], np.cumsum(g.n)]).astype(np.int64)
    # x_0, then (dense) the slacks of the inequality global rows
    T0, off0, ub0 = _var_map(g.lo[xo[-1]:], g.up[xo[-1]:])
    gslk = {}
    if dense:
        for k in range(g.ng):
            if g.dg[k] != g.fg[k]:
                gslk[k] = (T0.shape[1] + len(gslk),) + _slack_col(g.dg[k], g.fg[k])
        T0 = np.hstack([T0, np.zeros((n0, len(gslk)))])
    n0s = T0.shape[1]
    ub0_all = np.concatenate([ub0, np.full(n0s - n0, np.inf)])
    for k, (col, _, _, ubk) in gslk.items():
        ub0_all[col] = ubk
    # per block: primary and split columns, then inequality slacks
    Tb, offb, cols, slk = [], [], [], []
    for i in range(N):
        Ti, oi, ubi = _var_map(g.lo[xo[i]:xo[i + 1]], g.up[xo[i]:xo[i + 1]])
        ub = list(np.concatenate([ubi, np.full(Ti.shape[1] - g.n[i], np.inf)]))
        rows = [(g.d[i][r], g.f[i][r]) for r in range(g.d[i].size)]
        if i < N - 1:
            rows += [(g.dl[i][r], g.fl[i][r]) for r in range(g.dl[i].size)]
        if i == 0:
            rows += [(g.d0[r], g.f0[r]) for r in range(g.d0.size)]
        sl = [_slack_col(dv, fv) for dv, fv in rows]
        ub += [s[2] for s in sl]
        Tb.append(Ti)
        offb.append(oi)
        cols.append(ub)
        slk.append(sl)
    # upper-bound slacks (none when the bounds stay bounds)
    nub = [0 if bounds else int(np.isfinite(np.asarray(cols[i])).sum()) for i in range(N)]
    nub0 = 0 if bounds else int(np.isfinite(ub0_all).sum())
    ncol = [len(cols[i]) + nub[i] + (nub0 if i == 0 else 0) for i in range(N)]
    Tfull = []
    for i in range(N):
        T = np.zeros((int(g.n[i]), ncol[i]))
        T[:, :Tb[i].shape[1]] = Tb[i]
        Tfull.append(T)

    A, C, bs = [], [], []
    for i in range(N):
        nv = Tb[i].shape[1]               # primary + split columns
        mi = g.d[i].size
        # equality rows
        Ai = [g.A[i] @ Tfull[i]]
        Ci = [g.C[i] @ T0]
        bi = [g.b[int(g.m[:i].sum()):int(g.m[:i + 1].sum())] - g.A[i] @ offb[i] - g.C[i] @ off0]
        # inequality rows: r(x) - t = 0  ->  r(x_std) - sgn t' = off_r + off_t
        Hi = g.H[i] @ Tfull[i]
        Gi = g.G[i] @ T0
        rhs = -(g.H[i] @ offb[i]) - g.G[i] @ off0
        for r in range(mi):
            sgn, toff, _ = slk[i][r]
            Hi[r, nv + r] -= sgn
            rhs[r] += toff
        Ai.append(Hi); Ci.append(Gi); bi.append(rhs)
        if i == 0 and g.d0.size:
            base = nv + mi + (g.dl[0].size if N > 1 else 0)
            H0 = np.zeros((g.d0.size, ncol[0]))
            G0 = g.G0 @ T0
            r0 = -(g.G0 @ off0)
            for r in range(g.d0.size):
                sgn, toff, _ = slk[0][mi + (g.dl[0].size if N > 1 else 0) + r]
                H0[r, base + r] = -sgn
                r0[r] += toff
            Ai.append(H0); Ci.append(G0); bi.append(r0)
        # upper-bound rows
        ubs = np.asarray(cols[i])
        fin = np.flatnonzero(np.isfinite(ubs)) if not bounds else np.zeros(0, dtype=np.int64)
        U = np.zeros((fin.size, ncol[i]))
        UC = np.zeros((fin.size, n0s))
        for q, col in enumerate(fin):
            U[q, col] = 1.0
            U[q, len(cols[i]) + q] = 1.0
        ur = ubs[fin]
        Ai.append(U); Ci.append(UC); bi.append(ur)
        if i == 0 and nub0:
            fin0 = np.flatnonzero(np.isfinite(ub0_all))
            U0 = np.zeros((nub0, ncol[0]))
            U0C = np.zeros((nub0, n0s))
            for q, col in enumerate(fin0):
                U0C[q, col] = 1.0
                U0[q, len(cols[0]) + nub[0] + q] = 1.0
            Ai.append(U0); Ci.append(U0C); bi.append(ub0_all[fin0])
        A.append(np.vstack(Ai)); C.append(np.vstack(Ci)); bs.append(np.concatenate(bi))

    FR, FL, F0rows, bl = [], [], [], []
    lo_ = np.concatenate([[0], np.cumsum(g.l)]).astype(np.int64)
    mb = int(g.m.sum())
    for j in range(N - 1):
        fr = [g.FR[j] @ Tfull[j]]
        fl = [g.FL[j] @ Tfull[j + 1]]
        F0j = g.F0[lo_[j]:lo_[j + 1]] if g.F0 is not None else np.zeros((int(g.l[j]), n0))
        f0 = [F0j @ T0]
        rhs = [g.b[mb + lo_[j]: mb + lo_[j + 1]] - g.FR[j] @ offb[j] - g.FL[j] @ offb[j + 1] - F0j @ off0]
        kr = g.KR[j] @ Tfull[j]
        kl = g.KL[j] @ Tfull[j + 1]
        rr = -(g.KR[j] @ offb[j]) - g.KL[j] @ offb[j + 1]
        nv, mi = Tb[j].shape[1], g.d[j].size
        for r in range(g.dl[j].size):
            sgn, toff, _ = slk[j][mi + r]
            kr[r, nv + mi + r] -= sgn
            rr[r] += toff
        fr.append(kr); fl.append(kl); f0.append(np.zeros((g.dl[j].size, n0s))); rhs.append(rr)
        FR.append(np.vstack(fr)); FL.append(np.vstack(fl)); F0rows.append(np.vstack(f0))
        bl.append(np.concatenate(rhs))

    # global rows (dense): r(x_std) [- sgn t'] = side - r(offsets) [+ offset of t]
    Wg = [[] for _ in range(N)]
    Wg0, bg = [], []
    if dense:
        for k in range(g.ng):
            for i in range(N):
                Wg[i].append(g.Wg[i][k] @ Tfull[i])
            w0 = g.Wg0[k] @ T0
            rhs = -sum(g.Wg[i][k] @ offb[i] for i in range(N)) - g.Wg0[k] @ off0
            if k in gslk:
                col, sgn, toff, _ = gslk[k]
                w0[col] -= sgn
                rhs += toff
            else:
                rhs += g.dg[k]
            Wg0.append(w0)
            bg.append(rhs)
        for q in range(0 if g.A0 is None else g.A0.shape[0]):
            for i in range(N):
                Wg[i].append(np.zeros(ncol[i]))
            Wg0.append(g.A0[q] @ T0)
            bg.append(g.b0[q] - g.A0[q] @ off0)

    ms = np.array([a.shape[0] for a in A], dtype=np.int64)
    ns = np.array(ncol, dtype=np.int64)
    ls = np.array([f.shape[0] for f in FR], dtype=np.int64)
    F0 = np.vstack(F0rows) if F0rows and any(np.any(f) for f in F0rows) else None
    b = np.concatenate(bs + bl + [np.asarray(bg, dtype=float)]) if (bs or bl or bg) else np.zeros(0)
    cs = [Tfull[i].T @ g.c[xo[i]:xo[i + 1]] for i in range(N)] + [T0.T @ g.c[xo[-1]:]]
    const = float(sum(g.c[xo[i]:xo[i + 1]] @ offb[i] for i in range(N)) + g.c[xo[-1]:] @ off0)
    inst = Instance(N=N, n0=n0s, m=ms, n=ns, l=ls, A=A, C=C, FR=FR, FL=FL, F0=F0, b=b,
                    c=np.concatenate(cs))
    if bg:
        inst.Wg = [np.array(Wg[i]).reshape(len(bg), ncol[i]) for i in range(N)]
        inst.Wg0 = np.array(Wg0).reshape(len(bg), n0s)
    if bounds:
        inst.ub = np.concatenate([np.asarray(cols[i], dtype=float) for i in range(N)] + [ub0_all])
    mp = StandardMap(T=Tfull + [T0], off=offb + [off0],
                     xoff_std=np.concatenate([[0], np.cumsum(ns)]).astype(np.int64), const=const)
    return inst, mp


def from_standard(mp: StandardMap, x_std: np.ndarray) -> np.ndarray:
    """The general-form x of a standard-form point."""
    N = len(mp.T) - 1
    parts = [mp.off[i] + mp.T[i] @ x_std[mp.xoff_std[i]:mp.xoff_std[i + 1]] for i in range(N)]
    parts.append(mp.off[N] + mp.T[N] @ x_std[mp.xoff_std[N]:])
    x = np.concatenate(parts)
    if mp.keep is not None:
        x = x[mp.keep]
    if mp.x0map is not None:
        e, E, s0 = mp.x0map
        x = np.concatenate([x[:s0], e + E @ x[s0:]])
    return x


def solve(g: GeneralInstance, stream=None, dense=False, x0_border=False, bounds=False,
          history=False, **opts):
    """Solve a general instance on the current HIP device.  Returns
    (x, objective, result) with x in the general form's variables and the
    result dictionary of the standard-form interior-point run (with history,
    also its per-iteration records under "history").  dense, x0_border: keep
    the global rows (and the x_0-only equality rows) in the border of the
    Schur complement; bounds: keep the upper bounds inside the iteration (see
    to_standard)."""
    from .ahlp import Problem
    inst, mp = to_standard(g, dense=dense, x0_border=x0_border, bounds=bounds)
    P = Problem(inst, stream=stream)
    try:
        xs, _, _, res = P.ipm(stream=stream, **opts)
        if history:
            res["history"] = P.history()
        x = from_standard(mp, xs.detach().cpu().numpy())
    finally:
        P.close()
    return x, float(g.c @ x), res
