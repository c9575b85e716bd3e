"""General arrowhead LPs (Sec. 3.2: inequality rows and variable bounds) in
the oracle: an exact reformulation into the standard form of Sec. 2.2 with
the arrowhead structure kept, then the oracle interior-point method.

Test infrastructure only (see package docstring).

The paper states the general form but derives its method without the
inequality rows and bounds.  This reformulation is the textbook one:
  * x = lo + x' for a finite lower bound, x = up - x' for an upper bound
    only, x = x+ - x- for a free variable (all new variables >= 0);
  * an inequality row d <= r(x) <= f becomes r(x) - t = 0 with a slack t of
    bounds [d, f], itself reformulated like a variable;
  * a finite upper bound u' left after the shift becomes a row x' + s = u';
  * a global row dg <= sum_i Wg_i x_i + Wg_0 x_0 <= fg is first written as a
    chain of partial sums s_i = s_{i-1} + Wg_i x_i (free variables of block i;
    s_1 includes Wg_0 x_0), one row in block 1 and one link row per pair; the
    last partial sum gets the sides [dg, fg], except for an equality, whose
    last link row (block row if N = 1) carries dg instead.
Chaining layout: block i's partial sums follow its own variables (global row
order); block 1's and every link pair's new rows follow their own equality
rows.
Before all that, equality rows on x_0 alone (A_0 x_0 = b_0, full row rank)
are eliminated: the basic entries B of x_0 (the first r of a column-pivoted QR
of A_0) are x_B = B^-1 (b_0 - A_0,N x_N), substituted into every row that
touches x_0; x_N remain the linking variables with their own bounds, and each
bounded x_B becomes an x_0-only inequality row on x_N (after the existing
ones).
Placement (the layout the GPU path uses too): block i's columns are its
variables, x- of its free variables, the slacks of its inequality rows, of
link pair i's inequality rows and (block 1) of the x_0-only rows, then the
upper-bound slacks of those columns in order (block 1: then those of x_0);
its rows are its equality rows, its inequality rows (block 1: then the x_0
rows) and the upper-bound rows; x_0 is its variables then x- of its free
ones; link pair j has its equality rows then its inequality rows.

Dense layer (``dense=True``; the HSCA dense layer of Sec. 4.1): global rows
are kept whole as global rows of the standard form (Wg_i x_i + ... + Wg_0 x_0
= b_G), not chained; the x_0-only equality rows are eliminated as above, or,
with ``x0_border=True``, kept whole as global rows too (Wg_i = 0).  An
inequality global row gets its slack t (bounds [dg, fg]) as a new linking
variable: Wg x - t = 0, t an x_0 column after x_0's own and x- columns, in
global row order; its upper-bound slack row (if both sides are finite) goes to
block 1 like any other x_0 column's.  Global rows of the standard form: those
of the general instance in order, then the x_0-only equality rows.

Bounds inside the iteration (``bounds=True``): the finite upper bounds left
after the shifts are not turned into rows x' + s = u'; the standard form keeps
them as upper bounds of its columns (Instance.ub, +inf elsewhere), which the
interior-point method handles with slacks and duals of its own
(oracle/bounded.py).  Everything else is laid out as above.

Built here row by row from the global rows of the general instance and a
list of standard columns per original variable.
"""
from __future__ import annotations

import numpy as np

from paper_2412_07731_amd.gen import GeneralInstance, Instance, general_matrices

from . import ipm


class _Cols:
    """Standard columns of one block (or x_0): each a (kind, payload) entry."""

    def __init__(self):
        self.kinds = []     # 'x', 'xm', 't', 's'
        self.ub = []        # bound of the column after the reformulation

    def add(self, kind, ub):
        self.kinds.append(kind)
        self.ub.append(ub)
        return len(self.kinds) - 1


def eliminate_x0(g: GeneralInstance):
    """x_0-only equality rows eliminated: (instance over x_N, basic indices,
    nonbasic indices, B^-1 b_0, B^-1 A_0,N)."""
    import scipy.linalg as sla
    n0 = g.n0
    _, _, perm = sla.qr(g.A0, pivoting=True)
    r = g.A0.shape[0]
    bas, non = list(perm[:r]), list(perm[r:])
    Bm = g.A0[:, bas]
    u = np.linalg.solve(Bm, g.b0)                 # x_B = u - V x_N
    V = np.linalg.solve(Bm, g.A0[:, non])

    def sub_cols(M):
        """M x_0 = M[:, non] x_N + M[:, bas] (u - V x_N): (new matrix, constant)."""
        MB = M[:, bas]
        return M[:, non] - MB @ V, MB @ u

    C, G = [], []
    b = g.b.copy()
    d, f = [], []
    mfirst = np.concatenate([[0], np.cumsum(g.m)]).astype(np.int64)
    for i in range(g.N):
        Ci, ci = sub_cols(g.C[i])
        C.append(Ci)
        b[mfirst[i]:mfirst[i + 1]] = b[mfirst[i]:mfirst[i + 1]] - ci
        Gi, gi = sub_cols(g.G[i])
        G.append(Gi)
        d.append(g.d[i] - gi)
        f.append(g.f[i] - gi)
    F0 = None
    if g.F0 is not None:
        F0, f0c = sub_cols(g.F0)
        b[int(mfirst[-1]):] = b[int(mfirst[-1]):] - f0c
    Wg0, dg, fg = g.Wg0, g.dg, g.fg
    if g.ng:
        Wg0, wc = sub_cols(g.Wg0)
        dg, fg = g.dg - wc, g.fg - wc
    xs = int(g.n.sum())
    G0rows, d0, f0 = [], [], []
    if g.G0.shape[0]:
        G0n, gc0 = sub_cols(g.G0)
        G0rows.append(G0n)
        d0.append(g.d0 - gc0)
        f0.append(g.f0 - gc0)
    for q, j in enumerate(bas):
        lo, up = g.lo[xs + j], g.up[xs + j]
        if np.isfinite(lo) or np.isfinite(up):
            # x_B,q = u_q - V_q x_N  in [lo, up]  ->  -V_q x_N in [lo - u_q, up - u_q]
            G0rows.append(-V[q:q + 1])
            d0.append(np.array([lo - u[q]]))
            f0.append(np.array([up - u[q]]))
    c0 = g.c[xs:]
    cB = c0[bas]
    out = GeneralInstance(
        N=g.N, n0=len(non), m=g.m, n=g.n, l=g.l, A=g.A, C=C, FR=g.FR, FL=g.FL, F0=F0, b=b,
        H=g.H, G=G, d=d, f=f,
        G0=np.vstack(G0rows) if G0rows else np.zeros((0, len(non))),
        d0=np.concatenate(d0) if d0 else np.zeros(0), f0=np.concatenate(f0) if f0 else np.zeros(0),
        KR=g.KR, KL=g.KL, dl=g.dl, fl=g.fl,
        c=np.concatenate([g.c[:xs], c0[non] - V.T @ cB]),
        lo=np.concatenate([g.lo[:xs], g.lo[xs:][non]]),
        up=np.concatenate([g.up[:xs], g.up[xs:][non]]),
        Wg=g.Wg, Wg0=Wg0, dg=dg, fg=fg)
    return out, bas, non, u, V


def chain(g: GeneralInstance):
    """Global rows as chains of partial sums: an equivalent general instance
    without global rows, and the positions of the original variables in it."""
    N, n0, ng = g.N, g.n0, g.ng
    xo = np.concatenate([[0], np.cumsum(g.n)]).astype(np.int64)
    # per block, the partial sums it holds: list of global row indices
    sums = [[k for k in range(ng) if i < N - 1 or g.dg[k] != g.fg[k]] for i in range(N)]
    pos = [{k: int(g.n[i]) + q for q, k in enumerate(sums[i])} for i in range(N)]
    nn = np.array([int(g.n[i]) + len(sums[i]) for i in range(N)], dtype=np.int64)

    def widen(X, i):
        Y = np.zeros((X.shape[0], int(nn[i])))
        Y[:, :X.shape[1]] = X
        return Y

    A = [widen(g.A[i], i) for i in range(N)]
    C = [g.C[i].copy() for i in range(N)]
    brows = []
    mfirst = np.concatenate([[0], np.cumsum(g.m)]).astype(np.int64)
    for i in range(N):
        brows.append(list(g.b[mfirst[i]:mfirst[i + 1]]))
    lfirst = int(mfirst[-1]) + np.concatenate([[0], np.cumsum(g.l)]).astype(np.int64)
    lrows = [list(g.b[lfirst[j]:lfirst[j + 1]]) for j in range(N - 1)]
    FR = [widen(g.FR[j], j) for j in range(N - 1)]
    FL = [widen(g.FL[j], j + 1) for j in range(N - 1)]
    F0 = None
    if g.F0 is not None:
        F0 = [g.F0[lfirst[j] - lfirst[0]:lfirst[j + 1] - lfirst[0]] for j in range(N - 1)]
    for k in range(ng):
        # block 1 row: s_{k,1} - Wg_1 x_1 - Wg_0 x_0 = 0, or Wg_1 x_1 + Wg_0 x_0 = dg
        row = np.zeros(int(nn[0]))
        if k in pos[0]:
            row[:int(g.n[0])] = -g.Wg[0][k]
            row[pos[0][k]] = 1.0
            rc = -g.Wg0[k] if n0 else np.zeros(0)
            rhs = 0.0
        else:
            row[:int(g.n[0])] = -g.Wg[0][k]
            rc = -g.Wg0[k] if n0 else np.zeros(0)
            rhs = -g.dg[k]
        A[0] = np.vstack([A[0], row])
        C[0] = np.vstack([C[0], rc.reshape(1, n0)])
        brows[0].append(rhs)
    for j in range(N - 1):
        for k in range(ng):
            fr = np.zeros(int(nn[j]))
            fl = np.zeros(int(nn[j + 1]))
            fr[pos[j][k]] = -1.0
            fl[:int(g.n[j + 1])] = -g.Wg[j + 1][k]
            if k in pos[j + 1]:
                fl[pos[j + 1][k]] = 1.0
                rhs = 0.0
            else:
                rhs = -g.dg[k]
            FR[j] = np.vstack([FR[j], fr])
            FL[j] = np.vstack([FL[j], fl])
            if F0 is not None:
                F0[j] = np.vstack([F0[j], np.zeros((1, n0))])
            lrows[j].append(rhs)
    lo, up, c, keep = [], [], [], []
    start = 0
    for i in range(N):
        own = slice(xo[i], xo[i + 1])
        lo.append(g.lo[own]); up.append(g.up[own]); c.append(g.c[own])
        keep.extend(range(start, start + int(g.n[i])))
        for k in sums[i]:
            last = i == N - 1
            lo.append(np.array([g.dg[k] if last else -np.inf]))
            up.append(np.array([g.fg[k] if last else np.inf]))
            c.append(np.zeros(1))
        start += int(nn[i])
    lo.append(g.lo[xo[-1]:]); up.append(g.up[xo[-1]:]); c.append(g.c[xo[-1]:])
    keep.extend(range(start, start + n0))
    b = np.concatenate([np.asarray(r, dtype=float) for r in brows] +
                       [np.asarray(r, dtype=float) for r in lrows])
    m = np.array([A[i].shape[0] for i in range(N)], dtype=np.int64)
    l = np.array([FR[j].shape[0] for j in range(N - 1)], dtype=np.int64)
    out = GeneralInstance(N=N, n0=n0, m=m, n=nn, l=l, A=A, C=C, FR=FR, FL=FL,
                          F0=np.vstack(F0) if F0 else None, b=b,
                          H=[widen(g.H[i], i) for i in range(N)], G=g.G, d=g.d, f=g.f, G0=g.G0,
                          d0=g.d0, f0=g.f0, KR=[widen(g.KR[j], j) for j in range(N - 1)],
                          KL=[widen(g.KL[j], j + 1) for j in range(N - 1)], dl=g.dl, fl=g.fl,
                          c=np.concatenate(c), lo=np.concatenate(lo), up=np.concatenate(up))
    return out, np.array(keep, dtype=np.int64)


def reformulate(g: GeneralInstance, dense=False, x0_border=False, bounds=False):
    """Standard-form Instance, and for every original variable its
    (offset, [(block or -1 for x_0, column, sign)]) so x can be recovered
    (global rows are chained first, unless dense; their partial sums are
    dropped from the list)."""
    if not (dense and x0_border) and g.A0 is not None and g.A0.shape[0]:
        h, bas, non, u, V = eliminate_x0(g)
        inst, var, const = reformulate(h, dense=dense, bounds=bounds)
        # x_0 entries: x_N,k as reformulated; x_B,q = u_q - V_q x_N
        xs = int(g.n.sum())
        full = list(var[:xs]) + [None] * g.n0
        for k, j in enumerate(non):
            full[xs + j] = var[xs + k]
        for q, j in enumerate(bas):
            off = u[q]
            terms = []
            for k in range(len(non)):
                okk, tk = var[xs + k]
                off -= V[q, k] * okk
                terms += [(blk, col, -V[q, k] * sgn) for blk, col, sgn in tk]
            full[xs + j] = (off, terms)
        return inst, full, const + 0.0
    if not dense and g.ng:
        gc, keep = chain(g)
        inst, var, const = reformulate(gc, bounds=bounds)
        return inst, [var[k] for k in keep], const
    N, n0 = g.N, g.n0
    xo = np.concatenate([[0], np.cumsum(g.n)]).astype(np.int64)
    nt = g.n_tot
    Aeq, beq, Ain, dv, fv = general_matrices(g)
    Aeq, Ain = Aeq.tocsr(), Ain.tocsr()

    def owner(k):
        for i in range(N):
            if xo[i] <= k < xo[i + 1]:
                return i
        return -1

    blocks = [_Cols() for _ in range(N)]
    x0c = _Cols()
    var = [None] * nt            # (offset, [(blk, col, sign)])
    # 1. the variables' own columns, block by block, then x_0
    for k in range(nt):
        blk = owner(k)
        cols = blocks[blk] if blk >= 0 else x0c
        lo, up = g.lo[k], g.up[k]
        if np.isfinite(lo):
            c = cols.add('x', up - lo)
            var[k] = (lo, [(blk, c, 1.0)])
        elif np.isfinite(up):
            c = cols.add('x', np.inf)
            var[k] = (up, [(blk, c, -1.0)])
        else:
            c = cols.add('x', np.inf)
            var[k] = (0.0, [(blk, c, 1.0)])
    # 2. the minus parts of free variables
    for k in range(nt):
        if not np.isfinite(g.lo[k]) and not np.isfinite(g.up[k]):
            blk = owner(k)
            cols = blocks[blk] if blk >= 0 else x0c
            c = cols.add('xm', np.inf)
            var[k][1].append((blk, c, -1.0))
    # inequality rows in the global order: blocks, x_0-only, links
    mi = [g.d[i].size for i in range(N)]
    li = [g.dl[j].size for j in range(N - 1)]
    mi0 = g.d0.size
    ineq_home = []               # block of each inequality row's slack
    for i in range(N):
        ineq_home += [i] * mi[i]
    ineq_home += [0] * mi0
    for j in range(N - 1):
        ineq_home += [j] * li[j]
    # 3. slacks, per block in the documented order: own rows, pair i rows, x_0 rows
    mfirst_eq = np.concatenate([[0], np.cumsum(g.m)]).astype(np.int64)
    first = np.concatenate([[0], np.cumsum(mi)]).astype(np.int64)
    lfirst = int(first[-1]) + mi0 + np.concatenate([[0], np.cumsum(li)]).astype(np.int64)
    slack = {}                   # inequality row -> (blk, col, sign, offset)
    for i in range(N):
        order = list(range(int(first[i]), int(first[i + 1])))
        if i < N - 1:
            order += list(range(int(lfirst[i]), int(lfirst[i + 1])))
        if i == 0:
            order += list(range(int(first[-1]), int(first[-1]) + mi0))
        for r in order:
            if np.isfinite(dv[r]):
                c = blocks[i].add('t', fv[r] - dv[r] if np.isfinite(fv[r]) else np.inf)
                slack[r] = (i, c, 1.0, dv[r])
            else:
                c = blocks[i].add('t', np.inf)
                slack[r] = (i, c, -1.0, fv[r])
    # global rows in the order of the general instance, then the x_0-only
    # equality rows: ('eq', row of Aeq) or ('in', row of Ain); the slacks of
    # the inequality ones are x_0 columns
    grows = []
    if g.ng:
        ge = int(mfirst_eq[-1]) + int(g.l.sum())
        gi = int(lfirst[-1])
        for k in range(g.ng):
            if g.dg[k] == g.fg[k]:
                grows.append(('eq', ge))
                ge += 1
            else:
                grows.append(('in', gi))
                gi += 1
        a0 = ge
    else:
        a0 = int(mfirst_eq[-1]) + int(g.l.sum())
    if g.A0 is not None and g.A0.shape[0]:
        grows += [('eq', a0 + q) for q in range(g.A0.shape[0])]
    for kind, r in grows:
        if kind == 'in':
            if np.isfinite(dv[r]):
                c = x0c.add('t', fv[r] - dv[r] if np.isfinite(fv[r]) else np.inf)
                slack[r] = (-1, c, 1.0, dv[r])
            else:
                c = x0c.add('t', np.inf)
                slack[r] = (-1, c, -1.0, fv[r])
    # 4. upper-bound slacks (rows), unless the bounds stay bounds
    ubrows = [[] for _ in range(N)]   # (column holder block, column) bounded
    for i in (range(N) if not bounds else []):
        bounded = [c for c, u in enumerate(blocks[i].ub) if np.isfinite(u)]
        for c in bounded:
            s = blocks[i].add('s', np.inf)
            ubrows[i].append((i, c, s, blocks[i].ub[c]))
    for c, u in enumerate(x0c.ub if not bounds else []):
        if np.isfinite(u):
            s = blocks[0].add('s', np.inf)
            ubrows[0].append((-1, c, s, u))

    ncol = [len(blocks[i].kinds) for i in range(N)]
    n0s = len(x0c.kinds)

    def std_row(csr, r):
        """Row r of a global matrix in standard columns: dict per block, x_0
        part, right-hand side shift."""
        parts = {}
        x0 = np.zeros(n0s)
        shift = 0.0
        for p in range(csr.indptr[r], csr.indptr[r + 1]):
            k, a = int(csr.indices[p]), float(csr.data[p])
            offk, terms = var[k]
            shift += a * offk
            for blk, c, sgn in terms:
                if blk < 0:
                    x0[c] += a * sgn
                else:
                    parts.setdefault(blk, np.zeros(ncol[blk]))[c] += a * sgn
        return parts, x0, shift

    Ab = [[] for _ in range(N)]
    Cb = [[] for _ in range(N)]
    bb = [[] for _ in range(N)]

    def put_block_row(i, parts, x0, rhs):
        row = parts.get(i, np.zeros(ncol[i]))
        for blk in parts:
            if blk != i:
                raise ValueError("block row touches another block")
        Ab[i].append(row)
        Cb[i].append(x0)
        bb[i].append(rhs)

    mfirst = np.concatenate([[0], np.cumsum(g.m)]).astype(np.int64)
    for i in range(N):
        for r in range(int(mfirst[i]), int(mfirst[i + 1])):
            parts, x0, sh = std_row(Aeq, r)
            put_block_row(i, parts, x0, beq[r] - sh)
        rows = list(range(int(first[i]), int(first[i + 1])))
        if i == 0:
            rows += list(range(int(first[-1]), int(first[-1]) + mi0))
        for r in rows:
            parts, x0, sh = std_row(Ain, r)
            blk, c, sgn, toff = slack[r]
            parts.setdefault(blk, np.zeros(ncol[blk]))[c] -= sgn
            put_block_row(i, parts, x0, toff - sh)
        for holder, c, s, u in ubrows[i]:
            row = np.zeros(ncol[i])
            x0 = np.zeros(n0s)
            if holder < 0:
                x0[c] = 1.0
            else:
                row[c] = 1.0
            row[s] = 1.0
            Ab[i].append(row)
            Cb[i].append(x0)
            bb[i].append(u)

    FR, FL, F0r, bl = [], [], [], []
    lofs = np.concatenate([[0], np.cumsum(g.l)]).astype(np.int64)
    meq = int(mfirst[-1])
    for j in range(N - 1):
        fr, fl, f0, rh = [], [], [], []
        rows = [('eq', meq + int(lofs[j]) + q) for q in range(int(g.l[j]))]
        rows += [('in', int(lfirst[j]) + q) for q in range(li[j])]
        for kind, r in rows:
            parts, x0, sh = std_row(Aeq if kind == 'eq' else Ain, r)
            if kind == 'in':
                blk, c, sgn, toff = slack[r]
                parts.setdefault(blk, np.zeros(ncol[blk]))[c] -= sgn
                rhs = toff - sh
            else:
                rhs = beq[r] - sh
            fr.append(parts.get(j, np.zeros(ncol[j])))
            fl.append(parts.get(j + 1, np.zeros(ncol[j + 1])))
            f0.append(x0)
            rh.append(rhs)
        FR.append(np.array(fr).reshape(len(rows), ncol[j]))
        FL.append(np.array(fl).reshape(len(rows), ncol[j + 1]))
        F0r.append(np.array(f0).reshape(len(rows), n0s))
        bl += rh

    Wg = [[] for _ in range(N)]
    Wg0, bg = [], []
    for kind, r in grows:
        parts, x0, sh = std_row(Aeq if kind == 'eq' else Ain, r)
        if kind == 'in':
            blk, c, sgn, toff = slack[r]
            x0[c] -= sgn
            rhs = toff - sh
        else:
            rhs = beq[r] - sh
        for i in range(N):
            Wg[i].append(parts.get(i, np.zeros(ncol[i])))
        Wg0.append(x0)
        bg.append(rhs)

    A = [np.array(Ab[i]).reshape(len(Ab[i]), ncol[i]) for i in range(N)]
    C = [np.array(Cb[i]).reshape(len(Cb[i]), n0s) for i in range(N)]
    F0 = np.vstack(F0r) if F0r and any(np.any(f) for f in F0r) else None
    # cost: c_k x_k = c_k off_k + sum c_k sgn x_std
    cstd = [np.zeros(ncol[i]) for i in range(N)] + [np.zeros(n0s)]
    const = 0.0
    for k in range(nt):
        offk, terms = var[k]
        const += g.c[k] * offk
        for blk, c, sgn in terms:
            cstd[blk if blk >= 0 else N][c] += g.c[k] * sgn
    inst = Instance(N=N, n0=n0s, m=np.array([a.shape[0] for a in A], dtype=np.int64),
                    n=np.array(ncol, dtype=np.int64),
                    l=np.array([f.shape[0] for f in FR], dtype=np.int64), A=A, C=C, FR=FR,
                    FL=FL, F0=F0, b=np.concatenate([np.concatenate([np.asarray(v) for v in bb])
                                                    if N else np.zeros(0), np.asarray(bl),
                                                    np.asarray(bg)]),
                    c=np.concatenate(cstd))
    if grows:
        inst.Wg = [np.array(Wg[i]).reshape(len(grows), ncol[i]) for i in range(N)]
        inst.Wg0 = np.array(Wg0).reshape(len(grows), n0s)
    if bounds:
        inst.ub = np.concatenate([np.asarray(blocks[i].ub, dtype=float) for i in range(N)]
                                 + [np.asarray(x0c.ub, dtype=float)])
    return inst, var, const


def recover(g: GeneralInstance, inst: Instance, var, x_std):
    """x of the general form from a standard-form point."""
    xo = np.concatenate([[0], np.cumsum(inst.n)]).astype(np.int64)
    x = np.empty(len(var))
    for k, (offk, terms) in enumerate(var):
        v = offk
        for blk, c, sgn in terms:
            v += sgn * x_std[(xo[blk] if blk >= 0 else xo[-1]) + c]
        x[k] = v
    return x


def solve(g: GeneralInstance, opts=None, dense=False, x0_border=False, bounds=False):
    """Oracle solve of a general instance: (x, objective, ipm result)."""
    inst, var, _ = reformulate(g, dense=dense, x0_border=x0_border, bounds=bounds)
    if bounds:
        from . import bounded
        r = bounded.solve(inst, opts)
    else:
        r = ipm.solve(inst, opts) if opts is not None else ipm.solve(inst)
    x = recover(g, inst, var, r.x)
    return x, float(g.c @ x), r
