"""Pins of the oracle's general-form path (oracle/general.py: inequality rows
and variable bounds reformulated into the standard arrowhead form, then the
oracle IPM), to things other than itself:

* the optimum of the untransformed general LP from SciPy's HiGHS (bounds,
  two-sided rows, global rows and x_0-only equality rows handed over as they
  are), objective within 1e-7 relative (both solvers stop at about 1e-8);
* the recovered x is feasible in the general form: equality rows,
  inequality sides and bounds, within 1e-7;
* a closed form: min c'x over sum x = s with 0 <= x <= u (and one free
  variable fixed by a second row) is filled greedily in cost order;
* planted mistakes (upper bounds dropped; a global row's chain without its
  x_0 part; the substitution of eliminated x_0 entries without its constant
  part) fail the HiGHS pin;
* the GPU path's reformulation (paper_2412_07731_amd.general, written
  separately) produces the same standard-form instance;
* the dense layer (global rows kept whole in the border of S, and with
  x0_border the x_0-only equality rows too) reaches HiGHS's optimum of the
  untransformed LP, and a dropped x_0 part of its global rows fails that pin.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

from oracle import general as og
from paper_2412_07731_amd import gen, general


def highs(g):
    Aeq, beq, Ain, dv, fv = gen.general_matrices(g)
    ff, fd = np.isfinite(fv), np.isfinite(dv)
    A_ub = sp.vstack([Ain[ff], -Ain[fd]])
    b_ub = np.concatenate([fv[ff], -dv[fd]])
    bounds = [(a if np.isfinite(a) else None, b if np.isfinite(b) else None)
              for a, b in zip(g.lo, g.up)]
    r = linprog(g.c, A_ub=A_ub, b_ub=b_ub, A_eq=Aeq, b_eq=beq, bounds=bounds, method="highs")
    assert r.status == 0
    return r.fun


def violation(g, x):
    Aeq, beq, Ain, dv, fv = gen.general_matrices(g)
    r = Ain @ x
    return max(float(np.max(np.abs(Aeq @ x - beq), initial=0.0)),
               float(np.max(np.maximum(dv - r, 0.0), initial=0.0)),
               float(np.max(np.maximum(r - fv, 0.0), initial=0.0)),
               float(np.max(np.maximum(g.lo - x, 0.0))), float(np.max(np.maximum(x - g.up, 0.0))))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_general_matches_highs(seed):
    g = gen.generate_general("g_small", seed)
    # every bound and row kind is present, global rows of both kinds included
    assert np.isinf(g.lo).any() and np.isfinite(g.up).any() and (np.isinf(g.lo) & np.isinf(g.up)).any()
    assert (g.dg == g.fg).any() and (g.dg != g.fg).any()
    assert g.A0 is not None and g.A0.shape[0] >= 1          # an x_0-only equality row
    assert g.F0 is not None and np.any(g.F0)                # link rows on x_0
    x, f, r = og.solve(g)
    assert r.status == "optimal"
    fh = highs(g)
    assert abs(f - fh) <= 1e-7 * max(1.0, abs(fh))
    assert violation(g, x) <= 1e-7


def _box_instance(c, u, s):
    """One block, two rows: sum of the first k variables = s (0 <= x <= u),
    and x_free - x_0 = 1 with x_free free and x_0 in [0, 0.5] of cost 1."""
    k = len(c)
    A = np.zeros((2, k + 1))
    A[0, :k] = 1.0
    A[1, k] = 1.0
    Cm = np.array([[0.0], [-1.0]])
    g = gen.GeneralInstance(
        N=1, n0=1, m=np.array([2]), n=np.array([k + 1]), l=np.zeros(0, dtype=np.int64),
        A=[A], C=[Cm], FR=[], FL=[], F0=None, b=np.array([s, 1.0]),
        H=[np.zeros((0, k + 1))], G=[np.zeros((0, 1))], d=[np.zeros(0)], f=[np.zeros(0)],
        G0=np.zeros((0, 1)), d0=np.zeros(0), f0=np.zeros(0), KR=[], KL=[], dl=[], fl=[],
        c=np.concatenate([c, [0.0], [1.0]]),
        lo=np.concatenate([np.zeros(k), [-np.inf], [0.0]]),
        up=np.concatenate([u, [np.inf], [0.5]]))
    return g


def test_closed_form_box_knapsack():
    rng = np.random.default_rng(5)
    c = rng.uniform(-1.0, 2.0, 7)
    u = rng.uniform(0.5, 1.5, 7)
    s = 0.6 * u.sum()
    g = _box_instance(c, u, s)
    x, f, r = og.solve(g)
    assert r.status == "optimal"
    # greedy fill in cost order (all of sum = s must be placed)
    xr = np.zeros(7)
    left = s
    for j in np.argsort(c):
        xr[j] = min(u[j], left)
        left -= xr[j]
    fref = float(c @ xr)          # x_0 = 0 is optimal (cost 1), x_free = 1
    assert abs(f - fref) <= 1e-7 * max(1.0, abs(fref))
    assert np.max(np.abs(x[:7] - xr)) <= 1e-6
    assert abs(x[7] - 1.0) <= 1e-6 and abs(x[8]) <= 1e-6


def test_planted_mistake_fails():
    g = gen.generate_general("g_small", 0)
    fh = highs(g)
    bad = gen.generate_general("g_small", 0)
    bad.up = np.where(np.isfinite(bad.lo), np.inf, bad.up)    # boxes lose their upper side
    x, f, r = og.solve(bad)
    assert r.status != "optimal" or abs(f - fh) > 1e-3 * max(1.0, abs(fh))


@pytest.mark.parametrize("seed", [0, 3])
def test_planted_x0_elimination_mistake_fails(monkeypatch, seed):
    """The elimination of x_0-only equality rows drops the constant part of
    the substitution (x_B = B^-1 b_0 - ...) from the block rows' right-hand
    sides: the HiGHS pin catches it."""
    g = gen.generate_general("g_small", seed)
    fh = highs(g)
    real = og.eliminate_x0

    def broken(gg):
        out, bas, non, u, V = real(gg)
        out.b = gg.b.copy()
        return out, bas, non, u, V

    monkeypatch.setattr(og, "eliminate_x0", broken)
    x, f, r = og.solve(g)
    assert r.status != "optimal" or abs(f - fh) > 1e-4 * max(1.0, abs(fh))


def test_planted_chain_mistake_fails(monkeypatch):
    """The chain of a global row loses its x_0 part: the HiGHS pin catches it."""
    g = gen.generate_general("g_small", 2)
    fh = highs(g)
    real = og.chain

    def broken(gg):
        out, keep = real(gg)
        out.C[0][-gg.ng:] = 0.0
        return out, keep

    monkeypatch.setattr(og, "chain", broken)
    x, f, r = og.solve(g)
    assert r.status != "optimal" or abs(f - fh) > 1e-4 * max(1.0, abs(fh))


@pytest.mark.parametrize("seed,dense,x0b", [(0, False, False), (1, False, False), (0, True, False),
                                            (1, True, False), (3, True, True), (1, True, True)])
def test_two_reformulations_agree(seed, dense, x0b):
    g = gen.generate_general("g_small", seed)
    a, mp = general.to_standard(g, dense=dense, x0_border=x0b)
    b, var, const = og.reformulate(g, dense=dense, x0_border=x0b)
    assert a.N == b.N and a.n0 == b.n0 and a.ng == b.ng
    assert np.array_equal(a.m, b.m) and np.array_equal(a.n, b.n) and np.array_equal(a.l, b.l)
    if dense:
        assert a.ng > 0
        assert np.allclose(a.Wg0, b.Wg0, rtol=0, atol=1e-12)
        for u, v in zip(a.Wg, b.Wg):
            assert u.shape == v.shape and np.allclose(u, v, rtol=0, atol=1e-12)
    for X, Y in [(a.A, b.A), (a.C, b.C), (a.FR, b.FR), (a.FL, b.FL)]:
        for u, v in zip(X, Y):
            assert u.shape == v.shape and np.allclose(u, v, rtol=0, atol=1e-12)
    assert (a.F0 is None) == (b.F0 is None)
    assert np.allclose(a.b, b.b, rtol=0, atol=1e-12) and np.allclose(a.c, b.c, rtol=0, atol=1e-12)
    assert abs(mp.const - const) <= 1e-12
    xs = np.random.default_rng(seed).uniform(0, 1, a.n_tot)
    assert np.allclose(general.from_standard(mp, xs), og.recover(g, b, var, xs), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed,x0_border", [(0, False), (1, False), (2, False), (3, False),
                                            (0, True), (1, True), (2, True), (3, True)])
def test_dense_layer_matches_highs(seed, x0_border):
    g = gen.generate_general("g_small", seed)
    inst, var, _ = og.reformulate(g, dense=True, x0_border=x0_border)
    # the global rows stay whole (no chained partial sums); with x0_border so
    # do the x_0-only equality rows (no eliminated x_0 entries)
    me0 = g.A0.shape[0]
    assert inst.ng == g.ng + (me0 if x0_border else 0)
    x0v = slice(g.n_tot - g.n0, g.n_tot)
    free0 = np.isinf(g.lo[x0v]) & np.isinf(g.up[x0v])
    if x0_border:
        assert inst.n0 == g.n0 + int(np.sum(g.dg != g.fg)) + int(np.sum(free0))
    else:
        assert inst.n0 < g.n0 + int(np.sum(g.dg != g.fg)) + int(np.sum(free0))
    x, f, r = og.solve(g, dense=True, x0_border=x0_border)
    assert r.status == "optimal"
    fh = highs(g)
    assert abs(f - fh) <= 1e-7 * max(1.0, abs(fh))
    assert violation(g, x) <= 1e-7


def test_planted_dense_layer_mistake_fails(monkeypatch):
    """The global rows lose their x_0 part (Wg_0, which also holds the slacks
    of the inequality global rows): the HiGHS pin catches it."""
    g = gen.generate_general("g_small", 1)
    fh = highs(g)
    real = og.reformulate

    def broken(gg, dense=False, x0_border=False, bounds=False):
        inst, var, const = real(gg, dense=dense, x0_border=x0_border, bounds=bounds)
        inst.Wg0 = np.zeros_like(inst.Wg0)
        return inst, var, const

    monkeypatch.setattr(og, "reformulate", broken)
    x, f, r = og.solve(g, dense=True)
    assert r.status != "optimal" or abs(f - fh) > 1e-4 * max(1.0, abs(fh))
