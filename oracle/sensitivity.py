"""Sensitivity of an interior-point end point to the LP data (b, c).

Test infrastructure only (see package docstring).

What it computes.  With the barrier parameter held fixed, the perturbed KKT
conditions of Sec. 2.3

    F(x, y, z; b, c) = [A'y + z - c;  A x - b;  x z - mu e] = 0,   x, z > 0,

define the central-path point (x, y, z) as a smooth function of (b, c).  Its
derivative follows from the implicit function theorem with the unreduced
Newton matrix K = [[0, A', I], [A, 0, 0], [Z, 0, X]] (rows: dual, primal,
complementarity; unknowns dx, dy, dz):

    K [dx; dy; dz] = [dc; db; 0].

Forward derivatives (jvp) are one Newton solve.  The gradient of a scalar
L(x, f) with f = c'x is one solve with K' (vjp): with g = [dL/dx + (dL/df) c;
0; 0] and K' w = g, dL/db = w_y and dL/dc = w_x + (dL/df) x.  As mu -> 0 at a
nondegenerate optimum these tend to the LP sensitivities df/db = y*,
df/dc = x*, dx*/db = A_B^-1 on the basis (0 elsewhere) and dx*/dc = 0.

Functions
  kt_residual     g - K' w
  vjp_dense       K'^-1 g by dense LU of K' (tiny instances)
  vjp_block       K'^-1 g with the block factorization, through the scaling
                  identity K' = diag(I, I, Z^-1) K diag(I, I, Z)
  jvp             K^-1 [dc; db; 0] with the block solve, refined on K
  central_path    Newton on F = 0 for given (b, c, mu), to machine precision
  grad_objective  (df/db, df/dc) of f = c'x(b, c) from one vjp
"""
from __future__ import annotations

import numpy as np

from . import dense_kkt, lp, newton


def _inf(*vs):
    return max((float(np.max(np.abs(v))) if v.size else 0.0) for v in vs)


def kt_residual(inst, x, z, g, w):
    """g - K' w with K' = [[0, A', Z], [A, 0, 0], [I, 0, X]]."""
    gx, gy, gz = g
    wx, wy, wz = w
    return (gx - (lp.rmatvec(inst, wy) + z * wz),
            gy - lp.matvec(inst, wx),
            gz - (wx + x * wz))


def vjp_dense(inst, x, z, g):
    """K'^-1 g by dense LU of the transposed Newton matrix."""
    K = dense_kkt.newton_matrix(inst, x, z)
    gx, gy, gz = g
    w = np.linalg.solve(K.T, np.concatenate([gx, gy, gz]))
    n, m = gx.size, gy.size
    return w[:n], w[n:n + m], w[n + m:]


def vjp_block(inst, x, z, g, **kw):
    """K'^-1 g with the block factorization at (x, z).  The Newton matrix
    satisfies K' = S1 K S2 with S1 = diag(I, I, Z^-1), S2 = diag(I, I, Z)
    (check: S1 K S2 = [[0, A', Z], [A, 0, 0], [I, 0, X]]), so K' w = g is the
    Newton solve K d = (g_x, g_y, z g_z) followed by w = (dx, dy, dz / z).
    The Newton solve is refined on the unregularized K.  vjp_dense pins this
    on small instances.  Returns (w, backward error of the Newton solve)."""
    gx, gy, gz = g
    r = (np.asarray(gx, float), np.asarray(gy, float), z * np.asarray(gz, float))
    (dx, dy, dz), be = _solve_k(inst, x, z, r, **kw)
    return (dx, dy, dz / z), be


def _knorm(inst, x, z):
    rowabs, colabs = lp.abs_row_col_sums(inst)
    return lp.kkt_inf_norm(rowabs, colabs, x, z)


def k_residual(inst, x, z, r, d):
    """r - K d for the unreduced Newton matrix."""
    rx, ry, rz = r
    dx, dy, dz = d
    return (rx - (lp.rmatvec(inst, dy) + dz),
            ry - lp.matvec(inst, dx),
            rz - (z * dx + x * dz))


def jvp(inst, x, z, db, dc, **kw):
    """(dx, dy, dz) = K^-1 [dc; db; 0], block solve refined on K.  Returns
    (d, backward error)."""
    r = (np.asarray(dc, float), np.asarray(db, float), np.zeros_like(x))
    return _solve_k(inst, x, z, r, **kw)


def central_path(inst, x, y, z, mu, b, c, tol=1e-15, max_iter=30):
    """Newton's method on F(x, y, z; b, c) = 0 for fixed mu from (x, y, z),
    with a fraction-to-boundary step (0.9) to keep x, z > 0.  The scaled
    residual is max(|A'y + z - c|/(1+|c|), |A x - b|/(1+|b|), |x z - mu|/mu).
    Every Newton step is taken (the first step after a perturbation of (b, c)
    can raise the complementarity part, measured against the small mu, before
    the quadratic convergence sets in); it stops when the residual is <= tol
    or has not improved for three steps, and returns the best point."""
    x, y, z = (np.array(v, dtype=np.float64) for v in (x, y, z))
    bn, cn = 1.0 + _inf(b), 1.0 + _inf(c)

    def resid(x, y, z):
        return (lp.rmatvec(inst, y) + z - c, lp.matvec(inst, x) - b, x * z - mu)

    def size(F):
        return max(_inf(F[0]) / cn, _inf(F[1]) / bn, _inf(F[2]) / mu)

    F = resid(x, y, z)
    best = size(F)
    bx, by, bz = x, y, z
    stale = 0
    for _ in range(max_iter):
        if best <= tol or stale >= 3:
            break
        r = tuple(-v for v in F)
        d, _ = _solve_k(inst, x, z, r)
        dx, dy, dz = d
        a = 1.0
        for v, dv in ((x, dx), (z, dz)):
            neg = dv < 0
            if np.any(neg):
                a = min(a, 0.9 * float(np.min(-v[neg] / dv[neg])))
        x, y, z = x + a * dx, y + a * dy, z + a * dz
        F = resid(x, y, z)
        s = size(F)
        if s < best:
            best, bx, by, bz, stale = s, x, y, z, 0
        else:
            stale += 1
    return bx, by, bz, best


def _solve_k(inst, x, z, r, rho=1e-8, delta=1e-6, tol=1e-15, max_refine=30):
    f = newton.factor(inst, x, z, rho, delta)
    d = newton.solve(f, *r)
    kn, rn = _knorm(inst, x, z), _inf(*r)
    be = 0.0
    for _ in range(max_refine + 1):
        e = k_residual(inst, x, z, r, d)
        den = kn * _inf(*d) + rn
        be = _inf(*e) / den if den > 0 else 0.0
        if be <= tol:
            break
        c = newton.solve(f, *e)
        d = tuple(a + b for a, b in zip(d, c))
    return d, be


def grad_objective(inst, x, z, c, **kw):
    """(df/db, df/dc) of f = c'x at (x, z): one vjp with g = (c, 0, 0)."""
    g = (np.asarray(c, float), np.zeros(inst.m_tot), np.zeros_like(x))
    (wx, wy, _), be = vjp_block(inst, x, z, g, **kw)
    return wy, wx + x, be
