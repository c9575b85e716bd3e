"""Derivatives of the interior-point end point with respect to the LP data.

With the barrier parameter held at its final value, the KKT conditions of
Sec. 2.3,

    A'y + z = c,   A x = b,   x z = mu e,

define the end point (x, y, z) as a smooth function of (b, c).  By the implicit
function theorem its derivative is K^-1 [dc; db; 0] with K the Newton matrix
[[0, A', I], [A, 0, 0], [Z, 0, X]] at that point.  So

  * forward derivatives (jvp) are one Newton solve (ahlp_kkt_solve), and
  * the gradient of a scalar of (x, f = c'x) is one transposed solve
    (ahlp_lp_gradient) with g = (dL/dx + (dL/df) c, 0, 0):
    dL/db = w_y, dL/dc = w_x + (dL/df) x.

Both reuse one factorization at the end point.  At a nondegenerate optimum
these tend, as mu -> 0, to the LP sensitivities df/db = y*, df/dc = x*.

Everything runs in libahlp; this module only wires it into torch.autograd.
"""
from __future__ import annotations

import torch

from .ahlp import FP64

_IPM_DEFAULTS = dict(rho=1e-8, delta=1e-6)


class LPSolve(torch.autograd.Function):
    """(x, f) = LPSolve.apply(b, c, problem, opts): interior-point solve of the
    problem with right-hand side b and cost c (device float64 vectors), then a
    factorization at the end point that the backward pass reuses.  The problem
    handle is stateful: run backward before the next factor or solve on it.
    f is the library's objective c'x at the end point."""

    @staticmethod
    def forward(ctx, b, c, problem, opts):
        opts = dict(opts or {})
        b = b.detach().contiguous()
        c = c.detach().contiguous()
        problem.set_bc(b, c)
        ipm_opts = {k: v for k, v in opts.items() if k not in ("adjoint_refine", "adjoint_tol")}
        x, y, z, res = problem.ipm(**ipm_opts)
        if res["status"] != 0:
            raise RuntimeError(f"interior-point solve ended with {res['status_name']}")
        problem.factor(x, z, rho=opts.get("rho", _IPM_DEFAULTS["rho"]),
                       delta=opts.get("delta", _IPM_DEFAULTS["delta"]), precision=FP64)
        ctx.problem = problem
        ctx.max_refine = int(opts.get("adjoint_refine", 10))
        ctx.refine_tol = float(opts.get("adjoint_tol", 1e-12))
        f = torch.tensor(res["primal_obj"], dtype=torch.float64, device=x.device)
        return x, f

    @staticmethod
    def backward(ctx, gx, gf):
        gf = 0.0 if gf is None else float(gf)
        gx = None if gx is None else gx.contiguous()
        grad_b, grad_c, _ = ctx.problem.lp_gradient(gx, gf, max_refine=ctx.max_refine,
                                                     refine_tol=ctx.refine_tol)
        return grad_b, grad_c, None, None


def solve(problem, b, c, **opts):
    """Differentiable (x*, f*) for the LP with data (b, c)."""
    return LPSolve.apply(b, c, problem, opts)


def jvp(problem, db, dc, max_refine=10, refine_tol=1e-12):
    """(dx, dy, dz) = K^-1 [dc; db; 0] at the last factorization (forward
    derivative of the end point along (db, dc))."""
    rz = torch.zeros_like(dc)
    dx, dy, dz, _ = problem.solve(dc.contiguous(), db.contiguous(), rz, max_refine=max_refine,
                                  refine_tol=refine_tol)
    return dx, dy, dz
