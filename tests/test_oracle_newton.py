"""Pins of the oracle's block-elimination Newton solve (Alg. 2 / Alg. 3) to
things other than itself:

* brute force: a dense LU solve of the full unreduced Newton system of Sec. 2.3
  (and of the regularized augmented system) on tiny instances of many shapes;
* a library special case: at x = z = e without regularization the primal step
  for the right-hand side (0, r, 0) is the minimum-norm solution of A dx = r,
  which numpy.linalg.lstsq returns;
* the Schur complement: its inverse is the (y_L, y_G, x_0) block of the inverse
  of the whole augmented matrix (block elimination leaves that block
  unchanged); its zero pattern is App. A's (block tridiagonal plus border) and
  its nonzero count meets App. A's bound; its link part is positive definite
  and its border Schur complement negative definite, or, with global rows in
  the border (the dense layer of Sec. 4.1), of inertia (ng, n0).
"""
import numpy as np
import pytest

from oracle import dense_kkt, lp, newton
from paper_2412_07731_amd import gen


def shaped(N, m, n, l, n0, seed=0, dens=0.4, F0=False, ng=0):
    inst = gen.generate(dict(N=N, m=m, n=n, l=l, n0=n0, density=dens, ng=ng), seed)
    if F0:
        rng = np.random.default_rng(seed + 100)
        inst.F0 = rng.uniform(-1, 1, (int(inst.l.sum()), n0))
    return inst


def point(inst, seed=1, spread=(0.1, 2.0)):
    rng = np.random.default_rng(seed)
    n, m = inst.n_tot, inst.m_tot
    x = rng.uniform(*spread, n)
    z = rng.uniform(*spread, n)
    r = (rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(n))
    return x, z, r


SHAPES = [
    dict(N=1, m=6, n=12, l=0, n0=0),           # textbook normal equations
    dict(N=1, m=6, n=12, l=0, n0=3),
    dict(N=2, m=5, n=9, l=1, n0=0),
    dict(N=2, m=5, n=9, l=3, n0=2),
    dict(N=3, m=7, n=11, l=0, n0=4),           # no links: pure border
    dict(N=3, m=7, n=11, l=4, n0=1),
    dict(N=5, m=(3, 9), n="2m", l=(1, 3), n0=2),   # uneven blocks and pairs
    dict(N=8, m=32, n=64, l=4, n0=8),          # the tiny workload
    # global rows in the border (the dense layer)
    dict(N=1, m=6, n=12, l=0, n0=0, ng=2),     # border of global rows only
    dict(N=4, m=6, n=12, l=2, n0=0, ng=1),
    dict(N=3, m=7, n=11, l=4, n0=1, ng=3),
    dict(N=5, m=(3, 9), n="2m", l=(1, 3), n0=2, ng=4),
    dict(N=8, m=32, n=64, l=4, n0=8, ng=3),    # tiny_g
]


def rel(a, b):
    s = max(np.max(np.abs(b)), 1e-300)
    return np.max(np.abs(a - b)) / s


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("F0", [False, True])
def test_matches_dense_newton(shape, F0):
    if F0 and (shape["n0"] == 0 or shape["l"] == 0):
        pytest.skip("F0 needs links and linking variables")
    inst = shaped(**shape, F0=F0)
    x, z, r = point(inst)
    f = newton.factor(inst, x, z, 0.0, 0.0)
    d = newton.solve(f, *r)
    dd = dense_kkt.solve_newton(inst, x, z, *r)
    for a, b in zip(d, dd):
        assert rel(a, b) < 1e-11
    assert f.pivots == 0


@pytest.mark.parametrize("shape", SHAPES[3:])
def test_matches_dense_regularized(shape):
    inst = shaped(**shape, F0=True)
    x, z, r = point(inst, seed=4)
    rho, delta = 1e-3, 1e-2
    f = newton.factor(inst, x, z, rho, delta)
    d = newton.solve(f, *r)
    dd = dense_kkt.solve_regularized(inst, x, z, *r, rho, delta)
    for a, b in zip(d, dd):
        assert rel(a, b) < 1e-11


def test_ill_conditioned_point():
    """Late-IPM scaling: x and z spread over 1e-8..1e8."""
    inst = shaped(N=4, m=6, n=12, l=2, n0=2, seed=3)
    rng = np.random.default_rng(7)
    n = inst.n_tot
    x = 10.0 ** rng.uniform(-4, 4, n)
    z = 10.0 ** rng.uniform(-4, 4, n)
    r = (rng.standard_normal(n), rng.standard_normal(inst.m_tot), rng.standard_normal(n))
    f = newton.factor(inst, x, z, 0.0, 0.0)
    d = newton.solve(f, *r)
    K = dense_kkt.newton_matrix(inst, x, z)
    res = K @ np.concatenate(d) - np.concatenate(r)
    bk = np.max(np.abs(res)) / (np.max(np.abs(K).sum(1)) * np.max(np.abs(np.concatenate(d))) + np.max(np.abs(np.concatenate(r))))
    assert bk < 1e-12


@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[5], SHAPES[7]])
def test_min_norm_special_case(shape):
    """x = z = e, rho = delta = 0, rhs (0, r, 0): dx = A^+ r."""
    inst = shaped(**shape)
    n, m = inst.n_tot, inst.m_tot
    e = np.ones(n)
    r = np.random.default_rng(2).standard_normal(m)
    f = newton.factor(inst, e, e)
    dx, dy, dz = newton.solve(f, np.zeros(n), r, np.zeros(n))
    A = lp.full_matrix(inst).toarray()
    ls = np.linalg.lstsq(A, r, rcond=None)[0]
    assert rel(dx, ls) < 1e-11
    assert rel(dz, -dx) < 1e-14


def test_textbook_normal_equations():
    """N = 1, no links, no linking variables: dy solves (A D A') dy = ry + A D rx^
    with a Cholesky of the one normal matrix; checked here with a general LU."""
    inst = shaped(N=1, m=6, n=12, l=0, n0=0, seed=9)
    x, z, (rx, ry, rz) = point(inst, seed=3)
    f = newton.factor(inst, x, z)
    dx, dy, dz = newton.solve(f, rx, ry, rz)
    A = inst.A[0]
    Dg = x / z
    rhx = rx - rz / x
    dy_ref = np.linalg.solve(A @ np.diag(Dg) @ A.T, ry + A @ (Dg * rhx))
    assert rel(dy, dy_ref) < 1e-12


@pytest.mark.parametrize("shape", [SHAPES[3], SHAPES[6], SHAPES[7], SHAPES[10], SHAPES[11]])
def test_schur_is_block_of_augmented_inverse(shape):
    inst = shaped(**shape, F0=True)
    x, z, _ = point(inst, seed=5)
    rho, delta = 1e-4, 1e-3
    f = newton.factor(inst, x, z, rho, delta)
    S = newton.schur_matrix_dense(f)
    K = dense_kkt.augmented_matrix(inst, x, z, rho, delta)
    idx = dense_kkt.schur_indices(inst)
    Kinv = np.linalg.inv(K)[np.ix_(idx, idx)]
    assert rel(np.linalg.inv(S), Kinv) < 1e-9


def test_schur_structure_and_signs(tiny):
    inst = tiny
    x, z, _ = point(inst, seed=6)
    f = newton.factor(inst, x, z, 1e-8, 1e-6)
    S = newton.schur_matrix_dense(f)
    lo = inst.loff()
    nl = int(lo[-1])
    # App. A: pair blocks couple only to neighbouring pairs (and the border)
    pair = np.repeat(np.arange(inst.N - 1), inst.l)
    T = S[:nl, :nl]
    far = np.abs(pair[:, None] - pair[None, :]) > 1
    assert np.all(T[far] == 0)
    # nonzero bound of App. A (no global linking rows): met with equality here
    l = inst.l.astype(np.int64)
    bound = int(np.sum(l ** 2) + 2 * np.sum(l[:-1] * l[1:]) + 2 * np.sum(l) * inst.n0 + inst.n0 ** 2)
    assert np.count_nonzero(S) <= bound
    assert np.count_nonzero(S) == bound
    # quasi-definite: T > 0 and the border Schur complement < 0
    assert np.min(np.linalg.eigvalsh(T)) > 0
    Bs = S[nl:, nl:] - S[nl:, :nl] @ np.linalg.solve(T, S[:nl, nl:])
    assert np.max(np.linalg.eigvalsh(Bs)) < 0
    # symmetric
    assert np.array_equal(S, S.T)


@pytest.mark.parametrize("ng", [1, 3])
def test_dense_layer_structure_and_inertia(ng):
    """With global rows the border of S is [y_G, x_0]: T keeps App. A's pattern,
    E and S00 are dense, and the border Schur complement has exactly ng
    positive and n0 negative eigenvalues (quasi-definite); the border factor
    reproduces it as Lb diag(I, -I) Lb'."""
    inst = shaped(N=6, m=10, n=20, l=3, n0=4, seed=3, F0=True, ng=ng)
    x, z, _ = point(inst, seed=6)
    f = newton.factor(inst, x, z, 1e-8, 1e-6)
    S = newton.schur_matrix_dense(f)
    nl = int(inst.loff()[-1])
    pair = np.repeat(np.arange(inst.N - 1), inst.l)
    T = S[:nl, :nl]
    assert np.all(T[np.abs(pair[:, None] - pair[None, :]) > 1] == 0)
    assert np.min(np.linalg.eigvalsh(T)) > 0
    Bs = S[nl:, nl:] - S[nl:, :nl] @ np.linalg.solve(T, S[:nl, nl:])
    ev = np.linalg.eigvalsh(Bs)
    assert np.sum(ev > 0) == ng and np.sum(ev < 0) == inst.n0
    sig = np.concatenate([np.ones(ng), -np.ones(inst.n0)])
    assert rel((f.Lb * sig) @ f.Lb.T, Bs) < 1e-10
    assert np.all(np.triu(f.Lb, 1) == 0) and np.all(np.diag(f.Lb) > 0)
    assert rel(S, S.T) < 1e-15


def test_pivot_rule_on_rank_deficient_block():
    """A zero row in A_i makes M_i singular when delta = 0: the rule replaces
    that pivot (counted) and the direction still satisfies every other row."""
    inst = shaped(N=3, m=6, n=12, l=2, n0=2, seed=11)
    inst.A[1] = inst.A[1].copy()
    inst.A[1][2, :] = 0.0
    inst.C[1] = inst.C[1].copy()
    inst.C[1][2, :] = 0.0          # the whole constraint row is empty
    x, z, (rx, ry, rz) = point(inst, seed=8)
    yo = inst.yoff()
    ry[yo[1] + 2] = 0.0            # consistent right-hand side for the empty row
    f = newton.factor(inst, x, z, 0.0, 0.0)
    assert f.pivots == 1
    dx, dy, dz = newton.solve(f, rx, ry, rz)
    assert abs(dy[yo[1] + 2]) < 1e-50
    K = dense_kkt.newton_matrix(inst, x, z)
    res = K @ np.concatenate([dx, dy, dz]) - np.concatenate([rx, ry, rz])
    assert np.max(np.abs(res)) < 1e-10


def test_chol_rule_matches_lapack_and_column_loop():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((20, 20))
    M = X @ X.T + 1e-3 * np.eye(20)
    L, c = newton.chol_rule(M, 0.0)
    assert c == 0 and np.allclose(L @ L.T, M, atol=1e-12)
    # force the column loop with a threshold above one pivot
    L2, c2 = newton.chol_rule(M, 1e300)
    assert c2 == 20 and np.allclose(np.diag(L2), 1e64)


def test_nonfinite_and_nonpositive_rejected(tiny):
    n = tiny.n_tot
    x = np.ones(n)
    z = np.ones(n)
    x[3] = np.nan
    with pytest.raises(FloatingPointError):
        newton.factor(tiny, x, z)
    x[3] = 0.0
    with pytest.raises(FloatingPointError):
        newton.factor(tiny, x, z)


# -- planted mistakes: each plausible slip in the oracle must fail a pin ------

def _dense_pin_fails(inst):
    x, z, r = point(inst, seed=12)
    try:
        f = newton.factor(inst, x, z, 0.0, 0.0)
        d = newton.solve(f, *r)
    except (ValueError, IndexError):
        return True            # a mutant that cannot even run is caught too
    dd = dense_kkt.solve_newton(inst, x, z, *r)
    return max(rel(a, b) for a, b in zip(d, dd)) > 1e-6


def test_planted_mistakes_are_caught(monkeypatch):
    inst = shaped(N=4, m=5, n=10, l=2, n0=2, seed=13, F0=True)
    assert not _dense_pin_fails(inst)

    # 1. swapped left/right link blocks (wrong pair index)
    orig = newton.link_cols
    monkeypatch.setattr(newton, "link_cols", lambda ins, i: orig(ins, i)[::-1])
    assert _dense_pin_fails(inst)
    monkeypatch.undo()

    # 2. transposed operand in the back-solve
    monkeypatch.setattr(newton, "_ltsolve", newton._lsolve)
    assert _dense_pin_fails(inst)
    monkeypatch.undo()

    # 3. dropped F0 term (linking rows acting on x_0)
    F0 = inst.F0
    orig_factor = newton.factor

    def factor_noF0(ins, *a, **k):
        ins.F0 = None
        try:
            return orig_factor(ins, *a, **k)
        finally:
            ins.F0 = F0
    monkeypatch.setattr(newton, "factor", factor_noF0)
    assert _dense_pin_fails(inst)
    monkeypatch.undo()

    # 4. wrong sign of the x_0 diagonal block
    orig_solve = newton.schur_solve

    def flipped(f, sL, s0):
        f.Lb = f.Lb.copy()
        uL, u0 = orig_solve(f, sL, s0)
        return uL, -u0
    monkeypatch.setattr(newton, "schur_solve", flipped)
    assert _dense_pin_fails(inst)
    monkeypatch.undo()


def test_planted_mistakes_in_the_dense_layer(monkeypatch):
    inst = shaped(N=4, m=5, n=10, l=2, n0=2, seed=14, F0=True, ng=2)
    inst.Wg0 = np.random.default_rng(15).uniform(-1, 1, inst.Wg0.shape)
    assert not _dense_pin_fails(inst)

    # 1. global rows left out of the blocks' bordered columns
    monkeypatch.setattr(newton, "global_cols", lambda ins, i: np.zeros((0, int(ins.n[i]))))
    assert _dense_pin_fails(inst)
    monkeypatch.undo()

    # 2. the border taken as negative definite throughout (no + part)
    orig_bs = newton.border_solve

    def all_negative(f, t):
        ng = f.ng
        f.ng = 0
        try:
            return orig_bs(f, t)
        finally:
            f.ng = ng
    monkeypatch.setattr(newton, "border_solve", all_negative)
    assert _dense_pin_fails(inst)
    monkeypatch.undo()

    # 3. dropped x_0 part of the global rows (Wg_0)
    Wg0 = inst.Wg0
    orig_factor = newton.factor

    def factor_noWg0(ins, *a, **k):
        ins.Wg0 = np.zeros_like(Wg0)
        try:
            return orig_factor(ins, *a, **k)
        finally:
            ins.Wg0 = Wg0
    monkeypatch.setattr(newton, "factor", factor_noWg0)
    assert _dense_pin_fails(inst)
    monkeypatch.undo()


def test_late_iterate_forward_difference_is_conditioning():
    """Why the GPU parity of Newton directions is stated through backward
    errors and the forward-error bound they imply, not a bare elementwise
    1e-10: at a late interior-point iterate (mu ~ 5e-7) the oracle's refined
    block solve and a dense LU solve of the same unregularized Newton system
    both have small backward errors, yet differ element by element by far more
    than 1e-10, because K is ill-conditioned.  The difference is the one the
    two residuals imply: |d1 - d2| <= |K^-1| (|e1| + |e2|) componentwise."""
    from oracle import dense_kkt, ipm
    inst = gen.generate("tiny", 0)
    r = ipm.solve(inst, keep_iterates=True)
    h = min(r.history, key=lambda q: abs(np.log10(q["mu"] / 5e-7)))
    x, y, z = h["x"], h["y"], h["z"]
    rhs = (inst.c - lp.rmatvec(inst, y) - z, inst.b - lp.matvec(inst, x), -x * z)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    kn = lp.kkt_inf_norm(rowabs, colabs, x, z)
    st = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    d1, be1 = ipm.solve_refined(inst, newton.factor(inst, x, z, 1e-8, 1e-6), rhs, kn,
                                ipm.Options(), st)
    d2 = dense_kkt.solve_newton(inst, x, z, *rhs)
    K = dense_kkt.newton_matrix(inst, x, z)
    R = np.concatenate(rhs)
    D1, D2 = np.concatenate(d1), np.concatenate(d2)
    e1, e2 = R - K @ D1, R - K @ D2
    be2 = np.max(np.abs(e2)) / (kn * np.max(np.abs(D2)) + np.max(np.abs(R)))
    assert be1 <= 1e-9 and be2 <= 1e-9
    fwd = np.max(np.abs(D1 - D2)) / np.max(np.abs(D2))
    assert fwd > 1e-6                                  # far above 1e-10
    assert np.linalg.cond(K, np.inf) > 1e8
    eps = np.finfo(float).eps
    bound = np.abs(np.linalg.inv(K)) @ (np.abs(e1) + np.abs(e2)
                                        + 64 * eps * (np.abs(R) + np.abs(K) @ (np.abs(D1) + np.abs(D2))))
    assert np.all(np.abs(D1 - D2) <= 1.01 * bound)
