"""Upper bounds handled inside the interior-point iteration (oracle).

Test infrastructure only (see package docstring).

The LP of Sec. 2.2 with the bounds of Sec. 3.2 kept as bounds:

    min c'x   s.t.  Ax = b,  0 <= x <= u   (u_j = +inf: no upper bound)

An upper-bounded variable gets the slack s = u - x >= 0 with its dual w >= 0;
the optimality conditions become A'y + z - w = c, Ax = b, x + s = u, XZe = mu e,
SWe = mu e.  The Newton system in (dx, dy, dz, ds, dw) is

    A'dy + dz - dw = r_d      A dx = r_p      dx + ds = r_u
    Z dx + X dz = r_xz        W ds + S dw = r_sw

and eliminating ds = r_u - dx and dw = S^-1 (r_sw - W ds) leaves the Newton
system of Sec. 2.3 with one more diagonal in its (x, x) block,

    [[-Q, A', I], [A, 0, 0], [Z, 0, X]] (dx, dy, dz) = (r_d + S^-1 (r_sw - W r_u), r_p, r_xz),

Q = S^-1 W (zero for unbounded variables).  Its block elimination is the one of
Alg. 2 / Alg. 3 with D = (Z/X + Q + rho)^-1 (newton.factor's q), so the factor
and the solve of the standard form serve unchanged.  Refinement measures the
backward error on this system (the eliminated rows hold exactly by
construction).  Readings shared with the GPU driver:

  start   the standard start (x~, y~, z~ of ipm.starting_point's two solves);
          for bounded j: z_j = max(z~_j, 0), w_j = max(-z~_j, 0) (so z - w =
          z~), s_j = u_j - x~_j; the primal pair (x, s) and the dual pair
          (z, w) are each shifted by 1.5 times their most negative entry and
          then centred as in Mehrotra's heuristic, the sums taken over both.
  mu      (x'z + s'w) / (n + |U|), U the bounded variables.
  stop    relgap = |c'x - (b'y - u'w)| / max(1, |c'x|); pinf = max(|r_p|_inf /
          (1 + |b|_inf), |r_u|_inf / (1 + |u_U|_inf)); dinf = |c - A'y - z +
          w|_inf / (1 + |c|_inf).
  step    ratio tests over (x, s) for the primal and (z, w) for the dual step;
          mu_aff and sigma = (mu_aff / mu)^3 with both products; the
          corrector's products are sigma mu - XZe - dX dZ and sigma mu - SWe -
          dS dW.
  norm    |K|_inf = max(max_j (|A|_col,j + 1) + max q, max row sum of |A|,
          max(x + z)).
  Gondzio correctors are not combined with bounds.
"""
from __future__ import annotations

import numpy as np

from . import ipm, lp, newton


def bounded_mask(inst):
    u = getattr(inst, "ub", None)
    if u is None:
        return np.zeros(inst.n_tot, dtype=bool)
    return np.isfinite(u)


def newton_residual_q(inst, x, z, q, r, d):
    """e = r - K_q d for the reduced system above (K_q: the Newton matrix of
    Sec. 2.3 with -Q in its (x, x) block)."""
    rx, ry, rz = r
    dx, dy, dz = d
    ex = rx - (lp.rmatvec(inst, dy) + dz - q * dx)
    ey = ry - lp.matvec(inst, dx)
    ez = rz - (z * dx + x * dz)
    return ex, ey, ez


def reduced_rx(rd, ru, rsw, w, sinv):
    """The (x) right-hand side of the reduced system: r_d + S^-1 (r_sw - W r_u)."""
    return rd + sinv * (rsw - w * ru)


def recover_sw(U, ru, rsw, w, sinv, dx):
    """ds = r_u - dx and dw = S^-1 (r_sw - W ds) on the bounded variables."""
    ds = np.where(U, ru - dx, 0.0)
    return ds, sinv * (rsw - w * ds)


def solve_refined_q(inst, f, q, r, knorm, opts, stats):
    """newton.solve with refinement on K_q; returns (d, backward error)."""
    x, z = f.x, f.z
    d = newton.solve(f, *r)
    rnorm = ipm._inf(*r)
    steps = 0
    while True:
        e = newton_residual_q(inst, x, z, q, r, d)
        den = knorm * ipm._inf(*d) + rnorm
        be = ipm._inf(*e) / den if den > 0 else 0.0
        if be <= opts.refine_tol or steps >= opts.max_refine:
            break
        c = newton.solve(f, *e)
        d = tuple(a + b for a, b in zip(d, c))
        steps += 1
    stats["refine"] += steps
    stats["bkerr"] = max(stats["bkerr"], be)
    stats.setdefault("solves", []).append((be, steps))
    return d, be


def starting_point(inst, U, rowabs, colabs, opts, stats):
    """(x, y, z, s, w) by the start reading above; s = w = 0 off U."""
    n, m = inst.n_tot, inst.m_tot
    e = np.ones(n)
    f = newton.factor(inst, e, e, 0.0, 0.0)
    stats["pivots"] += f.pivots
    kn = lp.kkt_inf_norm(rowabs, colabs, e, e)
    d1, _ = ipm.solve_refined(inst, f, (np.zeros(n), inst.b.copy(), np.zeros(n)), kn, opts, stats)
    d2, _ = ipm.solve_refined(inst, f, (inst.c.copy(), np.zeros(m), np.zeros(n)), kn, opts, stats)
    xt, yt = d1[0], d2[1]
    zt = inst.c - lp.rmatvec(inst, yt)
    u = np.where(U, inst.ub, 0.0)
    z = np.where(U, np.maximum(zt, 0.0), zt)
    w = np.where(U, np.maximum(-zt, 0.0), 0.0)
    s = np.where(U, u - xt, 0.0)
    mp = min(float(np.min(xt)), float(np.min(s[U])) if U.any() else np.inf)
    md = min(float(np.min(z)), float(np.min(w[U])) if U.any() else np.inf)
    dp, dd = max(-1.5 * mp, 0.0), max(-1.5 * md, 0.0)
    x = xt + dp
    s = np.where(U, s + dp, 0.0)
    z = z + dd
    w = np.where(U, w + dd, 0.0)
    xz = float(x @ z) + float(s @ w)
    sx, sz = float(np.sum(x)) + float(np.sum(s)), float(np.sum(z)) + float(np.sum(w))
    cp = 0.5 * xz / sz if sz > 0 else 0.0
    cd = 0.5 * xz / sx if sx > 0 else 0.0
    x = x + cp
    s = np.where(U, s + cp, 0.0)
    z = z + cd
    w = np.where(U, w + cd, 0.0)
    if np.min(x) <= 0 or np.min(z) <= 0 or (U.any() and (np.min(s[U]) <= 0 or np.min(w[U]) <= 0)):
        x, z = x + 1.0, z + 1.0
        s, w = np.where(U, s + 1.0, 0.0), np.where(U, w + 1.0, 0.0)
    return x, yt.copy(), z, s, w


def _ratio_max(v, dv):
    neg = dv < 0
    if not np.any(neg):
        return np.inf
    return float(np.min(-v[neg] / dv[neg]))


def solve(inst, opts: ipm.Options = None, verbose=False, max_iter=None):
    """The interior-point method with the upper bounds inst.ub inside the
    iteration.  Returns an ipm.Result whose history entries also carry s and w
    norms; result.s, result.w are attached."""
    opts = opts or ipm.Options()
    if max_iter is not None:
        opts = ipm.Options(**{**opts.__dict__, "max_iter": max_iter})
    if opts.gondzio:
        raise ValueError("Gondzio correctors are not combined with bounds")
    U = bounded_mask(inst)
    nU = int(U.sum())
    u = np.where(U, inst.ub, 0.0)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    n = inst.n_tot
    stats = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    x, y, z, s, w = starting_point(inst, U, rowabs, colabs, opts, stats)
    bn = 1.0 + ipm._inf(inst.b)
    cn = 1.0 + ipm._inf(inst.c)
    un = 1.0 + (float(np.max(np.abs(u[U]))) if nU else 0.0)
    colmax = float(np.max(colabs + 1.0)) if colabs.size else 1.0
    rowmax = float(np.max(rowabs)) if rowabs.size else 0.0
    hist = []
    k = 0
    status = "maxiter"
    while True:
        rp = inst.b - lp.matvec(inst, x)
        ru = np.where(U, u - x - s, 0.0)
        rd = inst.c - lp.rmatvec(inst, y) - z + w
        mu = (float(x @ z) + float(s @ w)) / (n + nU)
        pobj, dobj = float(inst.c @ x), float(inst.b @ y) - float(u @ w)
        relgap = abs(pobj - dobj) / max(1.0, abs(pobj))
        pinf = max(ipm._inf(rp) / bn, ipm._inf(ru) / un)
        dinf = ipm._inf(rd) / cn
        if verbose:
            print(f"it {k:3d} mu {mu:.3e} gap {relgap:.3e} pinf {pinf:.3e} dinf {dinf:.3e}")
        if relgap <= opts.tol and pinf <= opts.tol and dinf <= opts.tol:
            status = "optimal"
            break
        if k >= opts.max_iter:
            break
        sinv = np.where(U, 1.0 / np.where(U, s, 1.0), 0.0)
        q = w * sinv
        f = newton.factor(inst, x, z, opts.rho, opts.delta, q=q)
        stats["pivots"] += f.pivots
        kn = max(colmax + (float(np.max(q)) if n else 0.0), rowmax, float(np.max(x + z)))

        def direction(rxz, rsw):
            rx = reduced_rx(rd, ru, rsw, w, sinv)
            d, be = solve_refined_q(inst, f, q, (rx, rp, rxz), kn, opts, stats)
            ds, dw = recover_sw(U, ru, rsw, w, sinv, d[0])
            return d, ds, dw, be

        da, dsa, dwa, be_a = direction(-x * z, -s * w)
        ap_aff = min(1.0, _ratio_max(x, da[0]), _ratio_max(s[U], dsa[U]) if nU else np.inf)
        ad_aff = min(1.0, _ratio_max(z, da[2]), _ratio_max(w[U], dwa[U]) if nU else np.inf)
        mu_aff = (float((x + ap_aff * da[0]) @ (z + ad_aff * da[2]))
                  + float((s + ap_aff * dsa) @ (w + ad_aff * dwa))) / (n + nU)
        sigma = (mu_aff / mu) ** 3
        smu = sigma * mu
        rxz = smu - x * z - da[0] * da[2]
        rsw = np.where(U, smu - s * w - dsa * dwa, 0.0)
        d, ds, dw, be = direction(rxz, rsw)
        ap = min(1.0, opts.eta * min(_ratio_max(x, d[0]), _ratio_max(s[U], ds[U]) if nU else np.inf))
        ad = min(1.0, opts.eta * min(_ratio_max(z, d[2]), _ratio_max(w[U], dw[U]) if nU else np.inf))
        hist.append(dict(k=k, mu=mu, relgap=relgap, pinf=pinf, dinf=dinf,
                         ap_aff=ap_aff, ad_aff=ad_aff, mu_aff=mu_aff,
                         sigma=sigma, ap=ap, ad=ad, bkerr_pred=be_a, bkerr=be, correctors=0))
        x = x + ap * d[0]
        s = np.where(U, s + ap * ds, 0.0)
        y = y + ad * d[1]
        z = z + ad * d[2]
        w = np.where(U, w + ad * dw, 0.0)
        k += 1
    r = ipm.Result(status=status, iterations=k, x=x, y=y, z=z, pobj=pobj, dobj=dobj,
                   relgap=relgap, pinf=pinf, dinf=dinf, mu=mu, pivots=stats["pivots"],
                   refine_steps=stats["refine"], max_bkerr=stats["bkerr"], history=hist,
                   solves=stats.get("solves", []))
    r.s, r.w = s, w
    return r
