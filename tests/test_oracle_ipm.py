"""Pins of the oracle's interior-point driver: the known optimum of every
generated LP (x* is unique, f* = c'x* = b'y*), the KKT conditions of Sec. 2.2,
an independent LP solver (scipy's HiGHS) on small cases, and the minimum-norm
property of Mehrotra's starting point.  The trajectory and iteration counts are
not printed in the paper; they are pinned only between the two implementations.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import ipm, lp
from paper_2412_07731_amd import gen


@pytest.mark.parametrize("seed", range(8))
def test_tiny_reaches_known_optimum(seed):
    inst = gen.generate("tiny", seed)
    r = ipm.solve(inst)
    assert r.status == "optimal"
    assert 5 <= r.iterations <= 20
    f = inst.fstar
    assert abs(r.pobj - f) <= 1e-7 * (1 + abs(f))
    assert np.max(np.abs(r.x - inst.xstar)) <= 1e-6 * (1 + np.max(np.abs(inst.xstar)))
    # KKT at the end: feasibility, positivity, small complementarity
    assert np.all(r.x > 0) and np.all(r.z > 0)
    assert r.relgap <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
    assert r.mu <= 1e-8 * (1 + abs(f))
    assert r.pivots == 0


@pytest.mark.parametrize("shape", [
    dict(N=3, m=5, n=11, l=2, n0=3, density=0.5),
    dict(N=4, m=(4, 8), n="2m", l=(1, 3), n0=2, density=0.4),
])
def test_matches_highs(shape):
    inst = gen.generate(shape, 21)
    A = lp.full_matrix(inst)
    ref = linprog(inst.c, A_eq=A, b_eq=inst.b, bounds=(0, None), method="highs")
    assert ref.status == 0
    r = ipm.solve(inst)
    assert r.status == "optimal"
    assert abs(r.pobj - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    assert abs(ref.fun - inst.fstar) <= 1e-9 * (1 + abs(inst.fstar))


def test_start_point_is_min_norm(tiny):
    """The first start-point solve returns A^+ b (the minimum-norm solution)."""
    from oracle import newton
    n = tiny.n_tot
    e = np.ones(n)
    f = newton.factor(tiny, e, e)
    dx = newton.solve(f, np.zeros(n), tiny.b, np.zeros(n))[0]
    ls = np.linalg.lstsq(lp.full_matrix(tiny).toarray(), tiny.b, rcond=None)[0]
    assert np.max(np.abs(dx - ls)) <= 1e-11 * np.max(np.abs(ls))


def test_max_iter_reported(tiny):
    r = ipm.solve(tiny, max_iter=2)
    assert r.status == "maxiter" and r.iterations == 2


def test_matvecs_are_adjoint(tiny):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(tiny.n_tot)
    y = rng.standard_normal(tiny.m_tot)
    assert abs(y @ lp.matvec(tiny, x) - x @ lp.rmatvec(tiny, y)) < 1e-10
    A = lp.full_matrix(tiny)
    assert np.allclose(A @ x, lp.matvec(tiny, x), atol=1e-13)


def test_kkt_norm_is_row_sum_norm(tiny):
    from oracle import dense_kkt
    rng = np.random.default_rng(3)
    x = rng.uniform(0.1, 3, tiny.n_tot)
    z = rng.uniform(0.1, 3, tiny.n_tot)
    rowabs, colabs = lp.abs_row_col_sums(tiny)
    K = dense_kkt.newton_matrix(tiny, x, z)
    assert abs(lp.kkt_inf_norm(rowabs, colabs, x, z) - np.max(np.abs(K).sum(axis=1))) < 1e-12
