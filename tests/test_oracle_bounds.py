"""Pins of the oracle's interior-point method with upper bounds inside the
iteration (oracle/bounded.py) to things other than itself:

* brute force: the direction of the reduced system (the Newton system of
  Sec. 2.3 with Q = W/S in its (x, x) block, ds and dw recovered by the
  elimination formulas) equals a dense LU solve of the whole Newton system in
  (dx, dy, dz, ds, dw), on shapes with and without global rows;
* planted mistakes (the sign of the bound term in the reduced right-hand side;
  Q left out of the factorization) fail that pin;
* the generator's known optimum (x*, f* with active and inactive upper
  bounds) and the KKT conditions;
* scipy's HiGHS on the same LPs, and on general-form instances whose bounds
  stay bounds (oracle.general with bounds=True) instead of becoming rows.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

from oracle import bounded, dense_kkt, lp, newton
from oracle import general as og
from paper_2412_07731_amd import gen

SHAPES = [
    dict(N=1, m=6, n=12, l=0, n0=0),
    dict(N=3, m=7, n=11, l=4, n0=1),
    dict(N=4, m=(4, 8), n="2m", l=(1, 3), n0=2),
    dict(N=5, m=(3, 9), n="2m", l=(1, 3), n0=2, ng=2),
]


def bounded_point(inst, seed):
    U = bounded.bounded_mask(inst)
    n, m = inst.n_tot, inst.m_tot
    rng = np.random.default_rng(seed)
    x, z = rng.uniform(0.1, 2, n), rng.uniform(0.1, 2, n)
    s = np.where(U, rng.uniform(0.1, 2, n), 0.0)
    w = np.where(U, rng.uniform(0.1, 2, n), 0.0)
    r = (rng.standard_normal(n), rng.standard_normal(m), np.where(U, rng.standard_normal(n), 0.0),
         rng.standard_normal(n), np.where(U, rng.standard_normal(n), 0.0))
    return U, x, z, s, w, r


def reduced_direction(inst, U, x, z, s, w, r, rx_fn=None, with_q=True):
    rd, rp, ru, rxz, rsw = r
    sinv = np.where(U, 1.0 / np.where(U, s, 1.0), 0.0)
    q = w * sinv
    f = newton.factor(inst, x, z, 0.0, 0.0, q=q if with_q else None)
    rx = (rx_fn or bounded.reduced_rx)(rd, ru, rsw, w, sinv)
    dx, dy, dz = newton.solve(f, rx, rp, rxz)
    ds, dw = bounded.recover_sw(U, ru, rsw, w, sinv, dx)
    return dx, dy, dz, ds, dw


def rel(a, b):
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


@pytest.mark.parametrize("shape", SHAPES)
def test_reduction_matches_dense_lu(shape):
    inst = gen.generate(dict(shape, density=0.4, ub_frac=0.5), 3)
    U, x, z, s, w, r = bounded_point(inst, 1)
    assert U.any()
    got = reduced_direction(inst, U, x, z, s, w, r)
    ref = dense_kkt.solve_newton_bounded(inst, x, z, s, w, U, *r)
    for a, b in zip(got, ref):
        assert rel(a, b) < 1e-12


def test_planted_mistakes_are_caught():
    inst = gen.generate(dict(N=4, m=(4, 8), n="2m", l=(1, 3), n0=2, density=0.4, ub_frac=0.5), 5)
    U, x, z, s, w, r = bounded_point(inst, 2)
    ref = dense_kkt.solve_newton_bounded(inst, x, z, s, w, U, *r)
    flipped = reduced_direction(inst, U, x, z, s, w, r,
                                rx_fn=lambda rd, ru, rsw, w_, si: rd - si * (rsw - w_ * ru))
    assert max(rel(a, b) for a, b in zip(flipped, ref)) > 1e-6
    noq = reduced_direction(inst, U, x, z, s, w, r, with_q=False)
    assert max(rel(a, b) for a, b in zip(noq, ref)) > 1e-6


@pytest.mark.parametrize("seed", range(4))
def test_known_optimum(seed):
    inst = gen.generate("tiny_b", seed)
    U = bounded.bounded_mask(inst)
    assert U.sum() > 100 and np.sum(inst.wstar > 0) > 20      # active and inactive bounds
    r = bounded.solve(inst)
    assert r.status == "optimal"
    f = inst.fstar
    assert abs(r.pobj - f) <= 1e-7 * (1 + abs(f))
    assert np.max(np.abs(r.x - inst.xstar)) <= 1e-6 * (1 + np.max(np.abs(inst.xstar)))
    assert np.all(r.x > 0) and np.all(r.z > 0) and np.all(r.s[U] > 0) and np.all(r.w[U] > 0)
    assert np.max(np.abs(r.x[U] + r.s[U] - inst.ub[U])) <= 1e-8 * (1 + np.max(inst.ub[U]))
    assert r.relgap <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8


def test_matches_highs():
    inst = gen.generate(dict(N=4, m=(4, 8), n="2m", l=(1, 3), n0=2, density=0.4, ub_frac=0.5), 21)
    A = lp.full_matrix(inst)
    bnds = [(0.0, u if np.isfinite(u) else None) for u in inst.ub]
    ref = linprog(inst.c, A_eq=A, b_eq=inst.b, bounds=bnds, method="highs")
    assert ref.status == 0
    r = bounded.solve(inst)
    assert r.status == "optimal"
    assert abs(r.pobj - ref.fun) <= 1e-7 * (1 + abs(ref.fun))


def _highs_general(g):
    Aeq, beq, Ain, dv, fv = gen.general_matrices(g)
    ff, fd = np.isfinite(fv), np.isfinite(dv)
    A_ub = sp.vstack([Ain[ff], -Ain[fd]])
    b_ub = np.concatenate([fv[ff], -dv[fd]])
    bnds = [(a if np.isfinite(a) else None, b if np.isfinite(b) else None) for a, b in zip(g.lo, g.up)]
    r = linprog(g.c, A_ub=A_ub, b_ub=b_ub, A_eq=Aeq, b_eq=beq, bounds=bnds, method="highs")
    assert r.status == 0
    return r.fun


@pytest.mark.parametrize("seed,dense", [(0, False), (1, False), (2, True), (3, True)])
def test_general_bounds_in_iteration_match_highs(seed, dense):
    g = gen.generate_general("g_small", seed)
    chained, _, _ = og.reformulate(g, dense=dense)
    inst, _, _ = og.reformulate(g, dense=dense, bounds=True)
    # the finite upper bounds stay bounds: fewer rows and columns than with
    # slack rows, the same count fewer of each
    nb = int(np.sum(np.isfinite(inst.ub)))
    assert nb > 0
    assert chained.m_tot - inst.m_tot == nb and chained.n_tot - inst.n_tot == nb
    x, f, r = og.solve(g, dense=dense, bounds=True)
    assert r.status == "optimal"
    fh = _highs_general(g)
    assert abs(f - fh) <= 1e-7 * max(1.0, abs(fh))
