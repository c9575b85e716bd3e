"""GPU parity of upper bounds inside the interior-point iteration (the bounds
of Sec. 3.2 kept as bounds): a bounded variable's slack s = u - x and dual w
are eliminated, which leaves the Newton system of Sec. 2.3 with -Q, Q = W/S,
in its (x, x) block, so the factorization and solve kernels serve unchanged.

Against the FP64 oracle (oracle/bounded.py):
* the direction of the Q-system (ahlp_kkt_factor_bounded + ahlp_kkt_solve)
  against the oracle's block elimination and against dense LU, with and
  without refinement;
* interior-point runs with the oracle's iteration count, objective and
  per-iterate backward errors (tiny_b seeds 0-3, mid_b), the generator's known
  optimum, and dual feasibility A'y + z - w = c with the library's w;
* general-form instances whose bounds stay bounds (g_small seeds 0-3,
  g_medium, g_large, and g_large through the dense layer too), FP32+refine,
  graph replays equal to the eager run, and the error for Gondzio correctors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import bounded, dense_kkt, lp, newton  # noqa: E402
from paper_2412_07731_amd import gen  # noqa: E402
from tests._parity import check_trajectory, golden  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_07731_amd import ahlp
    ahlp.lib()          # raises if the library is missing: no silent fallback
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=dev)


def H(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    s = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / s


@pytest.mark.parametrize("shape", [dict(N=3, m=7, n=11, l=4, n0=1),
                                   dict(N=8, m=32, n=64, l=4, n0=8),
                                   dict(N=6, m=(12, 40), n="2m", l=(1, 20), n0=5, ng=3)])
def test_q_system_direction(dev, shape):
    from paper_2412_07731_amd.ahlp import Problem
    print("case bounds direction", shape, flush=True)
    inst = gen.generate(dict(shape, density=0.4, ub_frac=0.5), 2)
    U = bounded.bounded_mask(inst)
    n, m = inst.n_tot, inst.m_tot
    rng = np.random.default_rng(3)
    x, z = rng.uniform(0.1, 2, n), rng.uniform(0.1, 2, n)
    q = np.where(U, rng.uniform(0.05, 5, n), 0.0)
    r = (rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(n))
    rho, delta = 1e-6, 1e-4
    P = Problem(inst)
    P.factor_bounded(T(x, dev), T(z, dev), T(q, dev), rho, delta)
    dx, dy, dz, _ = P.solve(*(T(v, dev) for v in r))
    f = newton.factor(inst, x, z, rho, delta, q=q)
    for a, b in zip((dx, dy, dz), newton.solve(f, *r)):
        assert rel(H(a), b) < 1e-10
    # refined on the unregularized Q-system: its backward error, and the
    # solution of dense LU of that system
    dx, dy, dz, be = P.solve(*(T(v, dev) for v in r), max_refine=5, refine_tol=1e-12)
    assert be <= 1e-12
    K = dense_kkt.newton_matrix(inst, x, z)
    K[:n, :n] -= np.diag(q)
    d = np.linalg.solve(K, np.concatenate(r))
    assert rel(np.concatenate([H(dx), H(dy), H(dz)]), d) < 1e-9
    P.close()


@pytest.mark.parametrize("config,seed", [("tiny_b", s) for s in range(4)] + [("mid_b", 0)])
def test_ipm_against_oracle(dev, config, seed):
    from paper_2412_07731_amd.ahlp import Problem
    print("case bounds ipm", config, seed, flush=True)
    inst = gen.generate(config, seed)
    g = golden(config, seed)
    P = Problem(inst)
    x, y, z, res = P.ipm()
    assert res["status"] == 0
    assert res["iterations"] == g["iterations"]
    assert abs(res["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
    assert abs(res["primal_obj"] - inst.fstar) <= 1e-7 * (1 + abs(inst.fstar))
    check_trajectory(P.history(), res, g, f"{config} seed {seed} bounds")
    s, w = (H(v) for v in P.bound_duals())
    U = bounded.bounded_mask(inst)
    xs = H(x)
    assert np.all(s[U] > 0) and np.all(w[U] > 0) and np.all(s[~U] == 0) and np.all(w[~U] == 0)
    assert np.max(np.abs(xs[U] + s[U] - inst.ub[U])) <= 1e-8 * (1 + np.max(inst.ub[U]))
    rd = inst.c - lp.rmatvec(inst, H(y)) - H(z) + w
    assert np.max(np.abs(rd)) <= 1e-7 * (1 + np.max(np.abs(inst.c)))
    P.close()


def test_ipm_fp32_refine(dev):
    from paper_2412_07731_amd.ahlp import FP32_REFINE, Problem
    print("case bounds fp32", flush=True)
    inst = gen.generate("mid_b", 0)
    g = golden("mid_b", 0)
    P = Problem(inst)
    x, y, z, res = P.ipm(precision=FP32_REFINE)
    assert res["status"] == 0 and res["fp32_iterations"] > 0
    assert abs(res["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
    P.close()


def test_graph_equals_eager(dev):
    from paper_2412_07731_amd.ahlp import Problem
    print("case bounds graph", flush=True)
    inst = gen.generate("mid_b", 0)
    P = Problem(inst)
    e = P.ipm()
    ge = [P.ipm(graph=1) for _ in range(2)]
    for g in ge:
        for a, b in zip(g[:3], e[:3]):
            assert torch.equal(a, b)
    P.close()


def test_gondzio_refused(dev):
    from paper_2412_07731_amd.ahlp import AHLPError, Problem
    inst = gen.generate("tiny_b", 0)
    P = Problem(inst)
    with pytest.raises(AHLPError):
        P.ipm(gondzio=2)
    P.close()


@pytest.mark.parametrize("config,seed,dense", [("g_small", s, False) for s in range(4)]
                         + [("g_medium", 0, False), ("g_large", 0, False), ("g_large", 0, True)])
def test_general_bounds_in_iteration(dev, config, seed, dense):
    from paper_2412_07731_amd import general
    print("case bounds general", config, seed, "dense" if dense else "", flush=True)
    g = gen.generate_general(config, seed)
    ref = golden(config, seed, dense=dense, bounds=True)
    x, f, res = general.solve(g, dense=dense, bounds=True, history=True)
    assert res["status"] == 0
    assert res["iterations"] == ref["iterations"]
    assert abs(f - ref["objective"]) <= 1e-8 * max(1.0, abs(ref["objective"]))
    # general instances are degenerate (free variables split into x+ - x-):
    # mu within 1e-4 (1e-3 in the last three iterations, mu below 1e-8) up to
    # the first refinement decision that differs
    check_trajectory(res["history"], res, ref, f"{config} seed {seed} bounds", mu_rtol_early=1e-4,
                     mu_rtol_late=1e-3)
    Aeq, beq, Ain, dv, fv = gen.general_matrices(g)
    rr = Ain @ x
    viol = max(float(np.max(np.abs(Aeq @ x - beq), initial=0.0)),
               float(np.max(np.maximum(dv - rr, 0.0), initial=0.0)),
               float(np.max(np.maximum(rr - fv, 0.0), initial=0.0)),
               float(np.max(np.maximum(g.lo - x, 0.0))), float(np.max(np.maximum(x - g.up, 0.0))))
    assert viol <= 1e-7
