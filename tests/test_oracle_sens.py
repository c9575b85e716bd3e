"""Pins of the oracle's sensitivity functions (oracle/sensitivity.py) to things
other than themselves, on the small nondegenerate instance:

* brute force: the block transposed solve equals a dense LU solve of K';
* the adjoint identity <g, K^-1 r> = <K'^-1 g, r> between the forward and the
  transposed solves (a transposed operand or a dropped scaling breaks it);
* central finite differences (h = 1e-6) of the mu-fixed central-path map,
  re-solved by Newton to machine precision, against the forward derivative;
* closed forms at a nondegenerate optimum (mu -> 0): df/db = y*, df/dc = x*,
  dx*/db = A_B^-1 db on the basis and 0 off it, dx*/dc = 0 (checked in
  absolute terms and as O(mu) on re-centring at mu / 100).
Planted mistakes (the z scaling of the transposed solve dropped; K used in
place of K') must fail the pins.
"""
import numpy as np
import pytest

from oracle import ipm, lp, sensitivity as sn
from paper_2412_07731_amd import gen


@pytest.fixture(scope="module")
def centred():
    """tiny_nd solved by the oracle IPM, then re-centred at mu = x'z/n."""
    inst = gen.generate("tiny_nd", 0)
    r = ipm.solve(inst)
    assert r.status == "optimal"
    mu = float(r.x @ r.z) / r.x.size
    x, y, z, res = sn.central_path(inst, r.x, r.y, r.z, mu, inst.b, inst.c)
    assert res <= 1e-14
    return inst, x, y, z, mu


def _rel(a, b):
    num = max(float(np.max(np.abs(u - v))) for u, v in zip(a, b))
    return num / max(float(np.max(np.abs(v))) for v in b)


def _g(inst, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(inst.n_tot), rng.standard_normal(inst.m_tot),
            rng.standard_normal(inst.n_tot))


@pytest.mark.parametrize("seed", [1, 2])
def test_vjp_block_matches_dense_lu(centred, seed):
    inst, x, y, z, mu = centred
    g = _g(inst, seed)
    wb, be = sn.vjp_block(inst, x, z, g)
    assert be <= 1e-14
    assert _rel(wb, sn.vjp_dense(inst, x, z, g)) <= 1e-10
    # residual of K' w = g itself
    e = sn.kt_residual(inst, x, z, g, wb)
    assert max(float(np.max(np.abs(v))) for v in e) <= 1e-9 * max(float(np.max(np.abs(v))) for v in g)


def test_adjoint_identity(centred):
    inst, x, y, z, mu = centred
    rng = np.random.default_rng(3)
    g = _g(inst, 4)
    db, dc = rng.standard_normal(inst.m_tot), rng.standard_normal(inst.n_tot)
    (dx, dy, dz), _ = sn.jvp(inst, x, z, db, dc)
    (wx, wy, wz), _ = sn.vjp_block(inst, x, z, g)
    lhs = g[0] @ dx + g[1] @ dy + g[2] @ dz
    rhs = wx @ dc + wy @ db
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_jvp_matches_central_differences(centred):
    inst, x, y, z, mu = centred
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(2):
        db = rng.standard_normal(inst.m_tot) * 1e-3 * np.linalg.norm(inst.b)
        dc = rng.standard_normal(inst.n_tot) * 1e-3 * np.linalg.norm(inst.c)
        (dx, dy, dz), _ = sn.jvp(inst, x, z, db, dc)
        xp, yp, zp, rp = sn.central_path(inst, x, y, z, mu, inst.b + h * db, inst.c + h * dc)
        xm, ym, zm, rm = sn.central_path(inst, x, y, z, mu, inst.b - h * db, inst.c - h * dc)
        assert max(rp, rm) <= 1e-14
        assert _rel([(xp - xm) / (2 * h), (yp - ym) / (2 * h)], [dx, dy]) <= 1e-6


def test_closed_forms_at_nondegenerate_optimum(centred):
    inst, x, y, z, mu = centred
    gb, gc, be = sn.grad_objective(inst, x, z, inst.c)
    assert np.max(np.abs(gb - inst.ystar)) <= 1e-6 * np.max(np.abs(inst.ystar))
    assert np.max(np.abs(gc - inst.xstar)) <= 1e-6 * np.max(np.abs(inst.xstar))
    # dx*/db = A_B^-1 db on the basis, 0 off it; dx*/dc = 0
    rng = np.random.default_rng(6)
    db = rng.standard_normal(inst.m_tot)
    (dx, _, _), _ = sn.jvp(inst, x, z, db, np.zeros(inst.n_tot))
    xo, _, _ = lp.offsets(inst)
    cols = np.concatenate([xo[i] + inst.basis[i] for i in range(inst.N)])
    AB = lp.full_matrix(inst).toarray()[:, cols]
    ref = np.zeros(inst.n_tot)
    ref[cols] = np.linalg.solve(AB, db)
    assert np.max(np.abs(dx - ref)) <= 1e-6 * np.max(np.abs(ref))
    # dx*/dc -> 0: absolute size, and O(mu) (re-centred at mu / 100)
    dc = rng.standard_normal(inst.n_tot)
    (dxc, _, _), _ = sn.jvp(inst, x, z, np.zeros(inst.m_tot), dc)
    big = np.max(np.abs(dxc))
    assert big <= 1e-4 * np.max(np.abs(dc))
    x2, y2, z2, r2 = sn.central_path(inst, x, y, z, mu * 1e-2, inst.b, inst.c)
    assert r2 <= 1e-14
    (dxc2, _, _), _ = sn.jvp(inst, x2, z2, np.zeros(inst.m_tot), dc)
    assert np.max(np.abs(dxc2)) <= 2e-2 * big


def test_planted_mistakes_fail(centred):
    inst, x, y, z, mu = centred
    g = _g(inst, 7)
    ref = sn.vjp_dense(inst, x, z, g)
    # the z scaling of the transposed solve dropped
    (dx, dy, dz), _ = sn._solve_k(inst, x, z, (g[0], g[1], z * g[2]))
    assert _rel((dx, dy, dz), ref) > 1e-3
    # K in place of K'
    (ex, ey, ez), _ = sn._solve_k(inst, x, z, g)
    assert _rel((ex, ey, ez), ref) > 1e-3
