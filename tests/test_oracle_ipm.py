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


@pytest.mark.parametrize("seed", range(4))
def test_gondzio_reaches_known_optimum(seed):
    """With up to two Gondzio correctors per iteration the end state is still
    the generator's optimum and no iteration count grows."""
    inst = gen.generate("tiny", seed)
    r0 = ipm.solve(inst)
    r2 = ipm.solve(inst, ipm.Options(gondzio=2))
    assert r2.status == "optimal"
    assert abs(r2.pobj - inst.fstar) <= 1e-7 * max(1.0, abs(inst.fstar))
    assert r2.iterations <= r0.iterations
    assert sum(h["correctors"] for h in r2.history) > 0


def test_gondzio_corrector_step(tiny):
    """One corrector at the first iteration: its correction solves the Newton
    system with right-hand side (0, 0, r) to dense-LU accuracy, the targets
    v + r lie in [beta_min, beta_max] sigma mu wherever v did not exceed the
    box, and a kept correction lengthens the smaller step by gamma delta_a."""
    from oracle import dense_kkt, newton
    inst = tiny
    opts = ipm.Options(gondzio=1)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    stats = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    x, y, z = ipm.starting_point(inst, rowabs, colabs, opts, stats)
    rp = inst.b - lp.matvec(inst, x)
    rd = inst.c - lp.rmatvec(inst, y) - z
    mu = float(x @ z) / inst.n_tot
    f = newton.factor(inst, x, z, opts.rho, opts.delta)
    kn = lp.kkt_inf_norm(rowabs, colabs, x, z)
    da, _ = ipm.solve_refined(inst, f, (rd, rp, -x * z), kn, opts, stats)
    ap_a, ad_a = ipm.ratio(x, da[0]), ipm.ratio(z, da[2])
    smu = (float((x + ap_a * da[0]) @ (z + ad_a * da[2])) / inst.n_tot / mu) ** 3 * mu
    d, _ = ipm.solve_refined(inst, f, (rd, rp, smu - x * z - da[0] * da[2]), kn, opts, stats)
    ap = min(1.0, opts.eta * ipm._ratio_max(x, d[0]))
    ad = min(1.0, opts.eta * ipm._ratio_max(z, d[2]))
    dn, ap_n, ad_n, kept = ipm.gondzio_corrector(inst, f, x, z, d, ap, ad, smu, kn, opts, stats)
    assert kept
    assert min(ap_n, ad_n) >= min(ap, ad) + opts.g_gamma * opts.g_delta_a
    at_p, at_d = min(1.0, ap + opts.g_delta_a), min(1.0, ad + opts.g_delta_a)
    v = (x + at_p * d[0]) * (z + at_d * d[2])
    lo, hi = opts.g_beta_min * smu, opts.g_beta_max * smu
    dc = [a - b for a, b in zip(dn, d)]
    # the correction's right-hand side, recovered from the Newton matrix
    K = dense_kkt.newton_matrix(inst, x, z)
    rhs = K @ np.concatenate(dc)
    n, m = inst.n_tot, inst.m_tot
    assert np.max(np.abs(rhs[:n + m])) <= 1e-8 * np.max(np.abs(rhs))
    r = rhs[n + m:]
    inside = v <= hi
    assert np.all(v[inside] + r[inside] >= lo * (1 - 1e-8))
    assert np.all(v[inside] + r[inside] <= hi * (1 + 1e-8))
    assert np.all(r >= -hi * (1 + 1e-8))
