"""Mehrotra predictor-corrector interior-point method (oracle).

Test infrastructure only (see package docstring).

The paper runs an infeasible primal-dual IPM with Mehrotra's predictor-corrector
scheme (Sec. 2, 2.3) and defers its details to the OOQP/PIPS literature.  The
constants and rules below are this implementation's reading; the GPU driver
uses the same ones.

  start   Mehrotra's heuristic: with x = z = e and no regularization solve for
          x~ = A'(AA')^-1 b and y~ = (AA')^-1 A c, z~ = c - A'y~; shift both to
          be nonnegative (1.5 times the most negative entry) and centre them.
  stop    relgap = |c'x - b'y| / max(1, |c'x|), pinf = |b - Ax|_inf / (1 + |b|_inf),
          dinf = |c - A'y - z|_inf / (1 + |c|_inf), all <= tol; the iteration
          count is the number of factorizations after the start point.
  step    predictor rhs (r_d, r_p, -XZe); alpha_aff by the ratio test;
          mu_aff = (x + a_p dx)'(z + a_d dz) / n; sigma = (mu_aff / mu)^3;
          corrector rhs (r_d, r_p, sigma mu e - XZe - dX_aff dZ_aff);
          a_p = min(1, eta a_p_max), a_d = min(1, eta a_d_max), eta = 0.99.
  refine  after every solve: e = r - K d with K the unregularized Newton matrix;
          backward error |e|_inf / (|K|_inf |d|_inf + |r|_inf); while it
          exceeds refine_tol and fewer than max_refine corrections were made,
          d += solve(e).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import lp, newton


@dataclass
class Options:
    tol: float = 1e-8
    max_iter: int = 100
    eta: float = 0.99
    rho: float = 1e-8
    delta: float = 1e-6
    max_refine: int = 5
    refine_tol: float = 1e-10
    # Gondzio's multiple centrality correctors after Mehrotra's corrector
    # (the paper's IPM extends Mehrotra's scheme with them; the constants are
    # readings): at most `gondzio` correctors per iteration
    gondzio: int = 0
    g_beta_min: float = 0.1
    g_beta_max: float = 10.0
    g_delta_a: float = 0.1
    g_gamma: float = 0.1


@dataclass
class Result:
    status: str
    iterations: int
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    pobj: float
    dobj: float
    relgap: float
    pinf: float
    dinf: float
    mu: float
    pivots: int = 0
    refine_steps: int = 0
    max_bkerr: float = 0.0
    history: list = field(default_factory=list)
    # (backward error, corrections) of every refined solve in call order: the
    # two start-point solves, then per iteration the predictor, the corrector
    # and any centrality correction
    solves: list = field(default_factory=list)


def newton_residual(inst, x, z, r, d):
    """e = r - K d for the unreduced Newton matrix of Sec. 2.3."""
    rx, ry, rz = r
    dx, dy, dz = d
    ex = rx - (lp.rmatvec(inst, dy) + dz)
    ey = ry - lp.matvec(inst, dx)
    ez = rz - (z * dx + x * dz)
    return ex, ey, ez


def _inf(*vs):
    return max((float(np.max(np.abs(v))) if v.size else 0.0) for v in vs)


def solve_refined(inst, f, r, knorm, opts, stats):
    """Newton solve with refinement; returns (d, backward error after the
    last correction).  stats["solves"] collects (backward error, corrections)
    per call, in call order."""
    x, z = f.x, f.z
    d = newton.solve(f, *r)
    rnorm = _inf(*r)
    steps = 0
    while True:
        e = newton_residual(inst, x, z, r, d)
        be = _inf(*e) / (knorm * _inf(*d) + rnorm) if (knorm * _inf(*d) + rnorm) > 0 else 0.0
        if be <= opts.refine_tol or steps >= opts.max_refine:
            break
        c = newton.solve(f, *e)
        d = tuple(a + b for a, b in zip(d, c))
        steps += 1
    stats["refine"] += steps
    stats["bkerr"] = max(stats["bkerr"], be)
    stats.setdefault("solves", []).append((be, steps))
    return d, be


def ratio(v, dv):
    """min(1, min over dv_j < 0 of -v_j / dv_j)."""
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    return min(1.0, float(np.min(-v[neg] / dv[neg])))


def starting_point(inst, rowabs, colabs, opts, stats):
    n, m = inst.n_tot, inst.m_tot
    e = np.ones(n)
    f = newton.factor(inst, e, e, 0.0, 0.0)
    stats["pivots"] += f.pivots
    kn = lp.kkt_inf_norm(rowabs, colabs, e, e)
    d1, _ = solve_refined(inst, f, (np.zeros(n), inst.b.copy(), np.zeros(n)), kn, opts, stats)
    d2, _ = solve_refined(inst, f, (inst.c.copy(), np.zeros(m), np.zeros(n)), kn, opts, stats)
    xt = d1[0]
    yt = d2[1]
    zt = inst.c - lp.rmatvec(inst, yt)
    xh = xt + max(-1.5 * float(np.min(xt)), 0.0)
    zh = zt + max(-1.5 * float(np.min(zt)), 0.0)
    xz = float(xh @ zh)
    sx, sz = float(np.sum(xh)), float(np.sum(zh))
    x0 = xh + (0.5 * xz / sz if sz > 0 else 0.0)
    z0 = zh + (0.5 * xz / sx if sx > 0 else 0.0)
    if np.min(x0) <= 0 or np.min(z0) <= 0:     # degenerate start: shift by one
        x0 = x0 + 1.0
        z0 = z0 + 1.0
    return x0, yt.copy(), z0


def solve(inst, opts: Options = None, verbose=False, max_iter=None, keep_iterates=False):
    """Runs the interior-point method from Mehrotra's starting point.  With
    keep_iterates every history entry also holds copies of the iterate
    (x, y, z) at the top of its iteration."""
    opts = opts or Options()
    if max_iter is not None:
        opts = Options(**{**opts.__dict__, "max_iter": max_iter})
    rowabs, colabs = lp.abs_row_col_sums(inst)
    n = inst.n_tot
    stats = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    x, y, z = starting_point(inst, rowabs, colabs, opts, stats)
    bn = 1.0 + _inf(inst.b)
    cn = 1.0 + _inf(inst.c)
    hist = []
    k = 0
    status = "maxiter"
    while True:
        rp = inst.b - lp.matvec(inst, x)
        rd = inst.c - lp.rmatvec(inst, y) - z
        mu = float(x @ z) / n
        pobj, dobj = float(inst.c @ x), float(inst.b @ y)
        relgap = abs(pobj - dobj) / max(1.0, abs(pobj))
        pinf, dinf = _inf(rp) / bn, _inf(rd) / cn
        if verbose:
            print(f"it {k:3d} mu {mu:.3e} gap {relgap:.3e} pinf {pinf:.3e} dinf {dinf:.3e}")
        if relgap <= opts.tol and pinf <= opts.tol and dinf <= opts.tol:
            status = "optimal"
            break
        if k >= opts.max_iter:
            break
        f = newton.factor(inst, x, z, opts.rho, opts.delta)
        stats["pivots"] += f.pivots
        kn = lp.kkt_inf_norm(rowabs, colabs, x, z)
        xz = x * z
        da, be_a = solve_refined(inst, f, (rd, rp, -xz), kn, opts, stats)
        ap_aff, ad_aff = ratio(x, da[0]), ratio(z, da[2])
        mu_aff = float((x + ap_aff * da[0]) @ (z + ad_aff * da[2])) / n
        sigma = (mu_aff / mu) ** 3
        rc = sigma * mu - xz - da[0] * da[2]
        d, be = solve_refined(inst, f, (rd, rp, rc), kn, opts, stats)
        ap = min(1.0, opts.eta * _ratio_max(x, d[0]))
        ad = min(1.0, opts.eta * _ratio_max(z, d[2]))
        ncorr = 0
        for _ in range(opts.gondzio):
            d, ap, ad, ok = gondzio_corrector(inst, f, x, z, d, ap, ad, sigma * mu, kn, opts, stats)
            if not ok:
                break
            ncorr += 1
        hist.append(dict(k=k, mu=mu, relgap=relgap, pinf=pinf, dinf=dinf,
                         ap_aff=ap_aff, ad_aff=ad_aff, mu_aff=mu_aff,
                         sigma=sigma, ap=ap, ad=ad, bkerr_pred=be_a, bkerr=be,
                         correctors=ncorr))
        if keep_iterates:
            hist[-1].update(x=x.copy(), y=y.copy(), z=z.copy())
        x = x + ap * d[0]
        y = y + ad * d[1]
        z = z + ad * d[2]
        k += 1
    return Result(status=status, iterations=k, x=x, y=y, z=z, pobj=pobj, dobj=dobj,
                  relgap=relgap, pinf=pinf, dinf=dinf, mu=mu, pivots=stats["pivots"],
                  refine_steps=stats["refine"], max_bkerr=stats["bkerr"], history=hist,
                  solves=stats.get("solves", []))


def gondzio_corrector(inst, f, x, z, d, ap, ad, smu, kn, opts, stats):
    """One multiple-centrality corrector (Gondzio).  Aim for step lengths
    longer by delta_a; at the trial point of those lengths the complementarity
    products v are moved into [beta_min, beta_max] sigma mu (a product above
    the box decreases by at most beta_max sigma mu); the correction solves the
    Newton system with right-hand side (0, 0, t - v).  It is kept when the
    smaller step length grows by at least gamma delta_a.  Returns the
    direction, the step lengths and whether the corrector was kept."""
    if ap >= 1.0 and ad >= 1.0:
        return d, ap, ad, False
    at_p = min(1.0, ap + opts.g_delta_a)
    at_d = min(1.0, ad + opts.g_delta_a)
    v = (x + at_p * d[0]) * (z + at_d * d[2])
    lo, hi = opts.g_beta_min * smu, opts.g_beta_max * smu
    r = np.maximum(np.clip(v, lo, hi) - v, -hi)
    n, m = x.size, d[1].size
    dc, _ = solve_refined(inst, f, (np.zeros(n), np.zeros(m), r), kn, opts, stats)
    dn = tuple(a + b for a, b in zip(d, dc))
    ap_n = min(1.0, opts.eta * _ratio_max(x, dn[0]))
    ad_n = min(1.0, opts.eta * _ratio_max(z, dn[2]))
    if min(ap_n, ad_n) >= min(ap, ad) + opts.g_gamma * opts.g_delta_a:
        return dn, ap_n, ad_n, True
    return d, ap, ad, False


def _ratio_max(v, dv):
    """Largest step keeping v + a dv >= 0 (infinite when dv >= 0)."""
    neg = dv < 0
    if not np.any(neg):
        return np.inf
    return float(np.min(-v[neg] / dv[neg]))
