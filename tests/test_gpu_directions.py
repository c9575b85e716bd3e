"""Newton directions of the FP64 path at interior-point states taken from the
oracle's own runs (mu near 1, 1e-2, 1e-4 and 1e-6), refined as in the
interior-point loop (at most 5 corrections, target 1e-10).

At each state the predictor's right-hand side (r_d, r_p, -XZe) is solved by
the library and by the oracle.  The checks:

* the library's backward error on the unregularized Newton system of
  Sec. 2.3, recomputed here from the returned direction with the oracle's
  residual, agrees with the one the library reports, and is at most
  max(1e-10, 10 eta_orc) (eta_orc: the oracle's on the same state; the
  oracle too misses 1e-10 where the system is nearly singular);
* element by element, the difference from the oracle's direction is within
  the forward-error bound that the two residuals imply:
  d_gpu - d_orc = K^-1 (e_orc - e_gpu) with e = r - K d, so
  |d_gpu - d_orc| <= |K^-1| (|e_gpu| + |e_orc|) component by component (dense
  K^-1, tiny), or in the infinity norm with an estimate of |K^-1| (larger).
  A bare 1e-10 on the forward difference would not hold: late in the run K
  has condition numbers of 1e9 and more, and two backward-stable solutions
  differ by up to 1e-2 (test_oracle_newton pins this on the oracle alone).

The relative forward difference |d_gpu - d_orc| / |d_orc| is printed for
every state.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import dense_kkt, ipm as oipm, lp, newton  # noqa: E402
from paper_2412_07731_amd import gen  # noqa: E402
from tests._parity import ETA, eta_bound  # noqa: E402

TARGETS = (1.0, 1e-2, 1e-4, 1e-6)
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_07731_amd import ahlp
    ahlp.lib()          # raises if the library is missing: no silent fallback
    return torch.device("cuda", 0)


def _inf(*vs):
    return max(float(np.max(np.abs(v))) if v.size else 0.0 for v in vs)


def oracle_states(inst, targets=TARGETS, max_iter=None):
    """Iterates of the oracle's run whose mu is closest (in log) to each target."""
    r = oipm.solve(inst, keep_iterates=True, max_iter=max_iter)
    mus = np.array([h["mu"] for h in r.history])
    out = []
    for t in targets:
        k = int(np.argmin(np.abs(np.log10(mus / t))))
        h = r.history[k]
        out.append((k, h["mu"], h["x"], h["y"], h["z"]))
    return out


def predictor_rhs(inst, x, y, z):
    return (inst.c - lp.rmatvec(inst, y) - z, inst.b - lp.matvec(inst, x), -x * z)


def solve_both(P, inst, x, z, r, dev, rowabs, colabs):
    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), device=dev)  # noqa: E731
    P.factor(T(x), T(z), 1e-8, 1e-6)
    dx, dy, dz, be_g = P.solve(*(T(v) for v in r), max_refine=5, refine_tol=1e-10)
    dg = tuple(t.cpu().numpy() for t in (dx, dy, dz))
    f = newton.factor(inst, x, z, 1e-8, 1e-6)
    kn = lp.kkt_inf_norm(rowabs, colabs, x, z)
    st = {"pivots": 0, "refine": 0, "bkerr": 0.0}
    do, be_o = oipm.solve_refined(inst, f, r, kn, oipm.Options(), st)
    eg = oipm.newton_residual(inst, x, z, r, dg)
    eo = oipm.newton_residual(inst, x, z, r, do)
    be_g2 = _inf(*eg) / (kn * _inf(*dg) + _inf(*r))
    return f, kn, dg, be_g, be_g2, do, be_o, eg, eo


def check_eta(label, be_g, be_g2, be_o):
    # the library's reported backward error is the one of the returned direction
    assert abs(be_g - be_g2) <= 1e-3 * be_g2 + 1e-18, (label, be_g, be_g2)
    assert be_g2 <= eta_bound(be_o), (label, be_g2, be_o)


@pytest.mark.parametrize("seed", [0, 3])
def test_directions_tiny(dev, seed):
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("tiny", seed)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    P = Problem(inst)
    try:
        for k, mu, x, y, z in oracle_states(inst):
            label = f"tiny seed {seed} iterate {k} mu {mu:.1e}"
            print("case", label, flush=True)
            r = predictor_rhs(inst, x, y, z)
            f, kn, dg, be_g, be_g2, do, be_o, eg, eo = solve_both(P, inst, x, z, r, dev, rowabs, colabs)
            check_eta(label, be_g, be_g2, be_o)
            K = dense_kkt.newton_matrix(inst, x, z)
            Kinv = np.abs(np.linalg.inv(K))
            G, O, R = np.concatenate(dg), np.concatenate(do), np.concatenate(r)
            # |e| as computed, plus the rounding of forming r - K d in FP64
            slack = 64 * EPS * (np.abs(R) + np.abs(K) @ (np.abs(G) + np.abs(O)))
            bound = Kinv @ (np.abs(np.concatenate(eg)) + np.abs(np.concatenate(eo)) + slack)
            diff = np.abs(G - O)
            fwd = float(np.max(diff) / np.max(np.abs(O)))
            print(f"  eta gpu {be_g2:.2e} oracle {be_o:.2e}  forward difference {fwd:.2e}  "
                  f"bound {float(np.max(bound) / np.max(np.abs(O))):.2e}", flush=True)
            assert np.all(diff <= 1.01 * bound), (label, float(np.max(diff / np.maximum(bound, 1e-300))))
    finally:
        P.close()


def kinv_inf_estimate(inst, f, x, z):
    """An estimate of |K^-1|_inf = |K^-T|_1 (Hager-Higham, scipy's onenormest)
    with the oracle's block solves: K^-1 v refined on K, and K^-T through the
    scaling identity K' = diag(I, I, Z^-1) K diag(I, I, Z)."""
    n, m = inst.n_tot, inst.m_tot
    rowabs, colabs = lp.abs_row_col_sums(inst)
    kn = lp.kkt_inf_norm(rowabs, colabs, x, z)
    opts = oipm.Options(max_refine=10, refine_tol=1e-14)

    def ksolve(v):
        st = {"pivots": 0, "refine": 0, "bkerr": 0.0}
        d, _ = oipm.solve_refined(inst, f, (v[:n], v[n:n + m], v[n + m:]), kn, opts, st)
        return np.concatenate(d)

    def kt_solve(v):     # K' w = v  <=>  K (wx, wy, z wz) = (vx, vy, z vz)
        u = v.copy()
        u[n + m:] *= z
        w = ksolve(u)
        w[n + m:] /= z
        return w

    N = 2 * n + m
    op = spla.LinearOperator((N, N), matvec=lambda v: kt_solve(np.ravel(v)),
                             rmatvec=lambda v: ksolve(np.ravel(v)), dtype=np.float64)
    return float(spla.onenormest(op, t=2))


def _normwise_case(P, inst, x, y, z, dev, label, rowabs, colabs):
    r = predictor_rhs(inst, x, y, z)
    f, kn, dg, be_g, be_g2, do, be_o, eg, eo = solve_both(P, inst, x, z, r, dev, rowabs, colabs)
    check_eta(label, be_g, be_g2, be_o)
    kinv = kinv_inf_estimate(inst, f, x, z)
    diff = max(float(np.max(np.abs(a - b))) for a, b in zip(dg, do))
    rounding = 64 * EPS * (kn * (_inf(*dg) + _inf(*do)) + 2 * _inf(*r))
    # the estimator is a lower bound, within a factor of 3 in practice
    bound = 3.0 * kinv * (_inf(*eg) + _inf(*eo) + rounding)
    fwd = diff / _inf(*do)
    print(f"  eta gpu {be_g2:.2e} oracle {be_o:.2e}  forward difference {fwd:.2e}  "
          f"bound {bound / _inf(*do):.2e}  |K^-1| ~ {kinv:.1e}", flush=True)
    assert diff <= bound, (label, diff, bound)


def test_directions_mid(dev):
    """N=64 blocks of 128 x 256 at 10%, 16 links per pair, 32 linking variables."""
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate(dict(N=64, m=128, n=256, l=16, n0=32, density=0.10), 0)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    P = Problem(inst)
    try:
        for k, mu, x, y, z in oracle_states(inst):
            label = f"mid iterate {k} mu {mu:.1e}"
            print("case", label, flush=True)
            _normwise_case(P, inst, x, y, z, dev, label, rowabs, colabs)
    finally:
        P.close()


def test_direction_n512_late(dev):
    """One late state of the N=512 workload (the oracle's iterate near mu = 1e-6)."""
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("n512", 0)
    rowabs, colabs = lp.abs_row_col_sums(inst)
    (k, mu, x, y, z), = oracle_states(inst, targets=(1e-6,))
    label = f"n512 iterate {k} mu {mu:.1e}"
    print("case", label, flush=True)
    P = Problem(inst)
    try:
        _normwise_case(P, inst, x, y, z, dev, label, rowabs, colabs)
    finally:
        P.close()
