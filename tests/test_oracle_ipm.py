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


@pytest.mark.parametrize("seed", range(4))
def test_global_rows_reach_known_optimum(seed):
    """Global linking rows kept in the border of S (the dense layer): the
    generated LP's known optimum and the KKT conditions."""
    inst = gen.generate("tiny_g", seed)
    assert inst.ng == 3
    r = ipm.solve(inst)
    assert r.status == "optimal"
    f = inst.fstar
    assert abs(r.pobj - f) <= 1e-7 * (1 + abs(f))
    assert np.max(np.abs(r.x - inst.xstar)) <= 1e-6 * (1 + np.max(np.abs(inst.xstar)))
    assert r.relgap <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
    assert r.pivots == 0


@pytest.mark.parametrize("shape", [
    dict(N=3, m=5, n=11, l=2, n0=3, density=0.5),
    dict(N=4, m=(4, 8), n="2m", l=(1, 3), n0=2, density=0.4),
    dict(N=4, m=(4, 8), n="2m", l=(1, 3), n0=2, density=0.4, ng=3),
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


def test_start_point_dual_is_least_squares(tiny):
    """The second start-point solve gives y~ = (AA')^-1 A c, the least-squares
    solution of A'y = c (A has full row rank), and the start keeps y0 = y~."""
    e = np.ones(tiny.n_tot)
    rowabs, colabs = lp.abs_row_col_sums(tiny)
    stats = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    x0, y0, z0 = ipm.starting_point(tiny, rowabs, colabs, ipm.Options(), stats)
    ls = np.linalg.lstsq(lp.full_matrix(tiny).toarray().T, tiny.c, rcond=None)[0]
    assert np.max(np.abs(y0 - ls)) <= 1e-11 * np.max(np.abs(ls))
    # x0 - x~ and z0 - z~ are multiples of e (the shift and the centring move
    # every entry by the same amount)
    xt = np.linalg.lstsq(lp.full_matrix(tiny).toarray(), tiny.b, rcond=None)[0]
    zt = tiny.c - lp.rmatvec(tiny, ls)
    for a, b in ((x0, xt), (z0, zt)):
        dv = a - b
        assert np.max(dv) - np.min(dv) <= 1e-10 * (1 + np.max(np.abs(a)))
    assert np.all(x0 > 0) and np.all(z0 > 0)


def _one_row_lp():
    """min x1 + 3 x2  s.t.  x1 + x2 = 2,  x >= 0 (one block, no links)."""
    return gen.Instance(N=1, n0=0, m=np.array([1]), n=np.array([2]), l=np.zeros(0, dtype=np.int64),
                        A=[np.array([[1.0, 1.0]])], C=[np.zeros((1, 0))], FR=[], FL=[], F0=None,
                        b=np.array([2.0]), c=np.array([1.0, 3.0]),
                        xstar=np.array([2.0, 0.0]), ystar=np.array([1.0]),
                        zstar=np.array([0.0, 2.0]), fstar=2.0)


def _newton_one_row(x, z, rd, rp, rz):
    """The Newton system of Sec. 2.3 for a single equality row a'x = b with
    a = e, solved by hand: dz = rd - dy e, x_i dz_i + z_i dx_i = rz_i, and
    sum dx = rp give one scalar equation for dy."""
    w = (rz - x * rd) / z
    dy = (rp - np.sum(w)) / np.sum(x / z)
    dz = rd - dy
    dx = (rz - x * dz) / z
    return dx, dy, dz


def test_mehrotra_worked_example():
    """Mehrotra's start and the first predictor-corrector iteration on a
    one-row LP, computed by hand.  Start: x~ = (1, 1), y~ = 2, z~ = (-1, 1);
    the shift adds 1.5 to z only (x~ >= 0); x'z = 3 after it, so the centring
    adds 0.5 * 3 / 3 = 0.5 to x and 0.5 * 3 / 2 = 0.75 to z:
    x0 = (1.5, 1.5), y0 = 2, z0 = (1.25, 3.25).  The iteration then takes the
    affine direction, its full-step ratio tests, mu_aff, sigma = (mu_aff/mu)^3,
    the corrector with sigma mu e - XZe - dXa dZa and steps 0.99 of the
    largest feasible ones."""
    inst = _one_row_lp()
    rowabs, colabs = lp.abs_row_col_sums(inst)
    stats = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    x0, y0, z0 = ipm.starting_point(inst, rowabs, colabs, ipm.Options(), stats)
    assert np.allclose(x0, [1.5, 1.5], rtol=0, atol=1e-12)
    assert np.allclose(y0, [2.0], rtol=0, atol=1e-12)
    assert np.allclose(z0, [1.25, 3.25], rtol=0, atol=1e-12)

    # first iteration by hand
    x, y, z = np.array([1.5, 1.5]), 2.0, np.array([1.25, 3.25])
    mu = x @ z / 2                                     # 3.375
    rp = 2.0 - x.sum()
    rd = np.array([1.0, 3.0]) - y - z
    dxa, dya, dza = _newton_one_row(x, z, rd, rp, -x * z)

    def step_max(v, dv):
        neg = dv < 0
        return np.inf if not neg.any() else float(np.min(-v[neg] / dv[neg]))

    apa, ada = min(1.0, step_max(x, dxa)), min(1.0, step_max(z, dza))
    mu_aff = (x + apa * dxa) @ (z + ada * dza) / 2
    sigma = (mu_aff / mu) ** 3
    dx, dy, dz = _newton_one_row(x, z, rd, rp, sigma * mu - x * z - dxa * dza)
    ap = min(1.0, 0.99 * step_max(x, dx))
    ad = min(1.0, 0.99 * step_max(z, dz))

    r = ipm.solve(inst, max_iter=1, keep_iterates=True)
    h = r.history[0]
    assert abs(h["mu"] - 3.375) <= 1e-12
    assert abs(h["mu_aff"] - mu_aff) <= 1e-9 * mu
    assert abs(h["sigma"] - sigma) <= 1e-8 * sigma
    assert abs(h["ap"] - ap) <= 1e-9 and abs(h["ad"] - ad) <= 1e-9
    assert np.allclose(r.x, x + ap * dx, rtol=0, atol=1e-9)
    assert np.allclose(r.y, [y + ad * dy], rtol=0, atol=1e-9)
    assert np.allclose(r.z, z + ad * dz, rtol=0, atol=1e-9)
    # and the method ends at the optimum (2, 0)
    full = ipm.solve(inst)
    assert full.status == "optimal" and abs(full.pobj - 2.0) <= 1e-8


@pytest.mark.parametrize("seed", [0, 5])
def test_predictor_backward_error_recorded(seed):
    """Every history entry carries the predictor's and the corrector's backward
    errors after refinement, each the largest |r - K d| / (|K| |d| + |r|) its
    solve reached: recomputed here from the kept iterate for the predictor."""
    from oracle import newton
    inst = gen.generate("tiny", seed)
    r = ipm.solve(inst, keep_iterates=True)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    for h in r.history[:4]:
        x, y, z = h["x"], h["y"], h["z"]
        rhs = (inst.c - lp.rmatvec(inst, y) - z, inst.b - lp.matvec(inst, x), -x * z)
        f = newton.factor(inst, x, z, 1e-8, 1e-6)
        kn = lp.kkt_inf_norm(rowabs, colabs, x, z)
        st = {"pivots": 0, "refine": 0, "bkerr": 0.0}
        d, be = ipm.solve_refined(inst, f, rhs, kn, ipm.Options(), st)
        e = ipm.newton_residual(inst, x, z, rhs, d)
        be2 = max(np.max(np.abs(v)) for v in e) / (kn * max(np.max(np.abs(v)) for v in d)
                                                  + max(np.max(np.abs(v)) for v in rhs))
        assert be == h["bkerr_pred"]
        assert abs(be2 - be) <= 1e-6 * be + 1e-20
    assert len(r.solves) == 2 + 2 * r.iterations
