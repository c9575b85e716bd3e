"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Stage by stage (block factors L_i and W_i = L_i^-1 B_i, the assembled Schur
complement), the Newton direction of Alg. 3 without and with refinement, and
the full interior-point run (identical iteration counts, objective within
1e-8).  Tolerances follow from FP64 rounding of the same block elimination
(different summation order only) and from the stated parity targets.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import dense_kkt, ipm as oipm, newton  # noqa: E402
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


def shaped(N, m, n, l, n0, seed=0, dens=0.4, F0=False):
    inst = gen.generate(dict(N=N, m=m, n=n, l=l, n0=n0, density=dens), seed)
    if F0:
        rng = np.random.default_rng(seed + 100)
        inst.F0 = rng.uniform(-1, 1, (int(inst.l.sum()), n0))
    return inst


def point(inst, seed=1, lo=0.1, hi=2.0):
    rng = np.random.default_rng(seed)
    n, m = inst.n_tot, inst.m_tot
    return (rng.uniform(lo, hi, n), rng.uniform(lo, hi, n),
            (rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(n)))


SHAPES = [
    dict(N=1, m=6, n=12, l=0, n0=0),
    dict(N=1, m=20, n=40, l=0, n0=3),
    dict(N=2, m=5, n=9, l=1, n0=0),
    dict(N=3, m=7, n=11, l=0, n0=4),
    dict(N=3, m=17, n=35, l=4, n0=1),             # ragged tiles (17 rows, 35 columns)
    dict(N=6, m=(12, 40), n="2m", l=(1, 20), n0=5),  # uneven blocks and pairs
    dict(N=8, m=32, n=64, l=4, n0=8),              # the tiny workload
    dict(N=40, m=48, n=96, l=16, n0=32),           # one-tile cyclic reduction, six levels
    dict(N=40, m=(40, 80), n="2m", l=(10, 32), n0=40),  # two-tile pairs (17..32 rows), six levels
    dict(N=33, m=(36, 60), n="2m", l=(17, 32), n0=64),  # two-tile pairs, full border
    dict(N=12, m=(48, 80), n="2m", l=(30, 40), n0=6),   # pairs over 32 rows: segmented chain
]


def ids(s):
    return "N{N}-m{m}-l{l}-n0{n0}".format(**s).replace(" ", "")


@pytest.mark.parametrize("shape", SHAPES, ids=[ids(s) for s in SHAPES])
def test_stages_and_direction(dev, shape):
    from paper_2412_07731_amd.ahlp import Problem
    F0 = shape["n0"] > 0 and shape["l"] != 0
    inst = shaped(**shape, F0=F0)
    print("case", ids(shape), flush=True)
    x, z, r = point(inst)
    rho, delta = 1e-6, 1e-4
    P = Problem(inst)
    P.factor(T(x, dev), T(z, dev), rho, delta)
    dx, dy, dz, _ = P.solve(*(T(v, dev) for v in r))
    torch.cuda.synchronize()
    f = newton.factor(inst, x, z, rho, delta)
    for i in sorted({0, inst.N // 2, inst.N - 1}):
        Lg, Wg = P.debug_block(i)
        assert rel(Lg, f.L[i]) < 1e-12, ("L", i)
        if f.W[i].size:
            assert rel(Wg, f.W[i]) < 1e-11, ("W", i)
    if inst.N > 1 or inst.n0 > 0:
        S = P.debug_schur()
        assert rel(S, newton.schur_matrix_dense(f)) < 1e-11
    d = newton.solve(f, *r)
    for a, b in zip((dx, dy, dz), d):
        assert rel(H(a), b) < 1e-10
    assert P.pivots() == 0
    P.close()


def test_direction_against_dense_lu(dev):
    """The GPU direction against a brute-force dense LU of the whole Newton system."""
    from paper_2412_07731_amd.ahlp import Problem
    inst = shaped(N=5, m=(3, 9), n="2m", l=(1, 3), n0=2, F0=True)
    x, z, r = point(inst, seed=4)
    P = Problem(inst)
    P.factor(T(x, dev), T(z, dev), 0.0, 0.0)
    d = P.solve(*(T(v, dev) for v in r))
    dd = dense_kkt.solve_newton(inst, x, z, *r)
    for a, b in zip(d[:3], dd):
        assert rel(H(a), b) < 1e-10
    P.close()


def test_refinement_reaches_backward_error(dev):
    """Ill-conditioned point (x, z over 1e-6..1e6): after refinement the
    backward error on the unregularized Newton system is <= 1e-10."""
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("tiny", 3)
    rng = np.random.default_rng(5)
    n, m = inst.n_tot, inst.m_tot
    x = 10.0 ** rng.uniform(-6, 6, n)
    z = 10.0 ** rng.uniform(-6, 6, n)
    r = (rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(n))
    P = Problem(inst)
    P.factor(T(x, dev), T(z, dev), 1e-8, 1e-6)
    dx, dy, dz, be = P.solve(*(T(v, dev) for v in r), max_refine=5, refine_tol=1e-10)
    K = dense_kkt.newton_matrix(inst, x, z)
    d = np.concatenate([H(dx), H(dy), H(dz)])
    rr = np.concatenate(r)
    true_be = np.max(np.abs(rr - K @ d)) / (np.max(np.abs(K).sum(1)) * np.max(np.abs(d)) + np.max(np.abs(rr)))
    assert be <= 1e-10 and true_be <= 1e-10
    P.close()


@pytest.mark.parametrize("seed", range(8))
def test_ipm_tiny_matches_oracle(dev, seed):
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("tiny", seed)
    g = golden("tiny", seed)
    P = Problem(inst)
    x, y, z, res = P.ipm()
    print("seed", seed, res["iterations"], res["primal_obj"], g["iterations"], g["pobj"], flush=True)
    assert res["status"] == 0
    assert res["iterations"] == g["iterations"]
    assert abs(res["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
    assert abs(res["primal_obj"] - inst.fstar) <= 1e-7 * (1 + abs(inst.fstar))
    assert np.max(np.abs(H(x) - inst.xstar)) <= 1e-6 * (1 + np.max(inst.xstar))
    check_trajectory(P.history(), res, g, f"tiny seed {seed}")
    P.close()


def test_determinism(dev):
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("tiny", 2)
    P = Problem(inst)
    a = [H(t) for t in P.ipm()[:3]]
    b = [H(t) for t in P.ipm()[:3]]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    P.close()


def test_error_paths(dev):
    from paper_2412_07731_amd import ahlp
    inst = gen.generate("tiny", 0)
    P = ahlp.Problem(inst)
    n, m = inst.n_tot, inst.m_tot
    zn, zm = torch.zeros(n, dtype=torch.float64, device=dev), torch.zeros(m, dtype=torch.float64, device=dev)
    with pytest.raises(ahlp.AHLPError) as e:
        P.solve(zn, zm, zn)
    assert e.value.code == -4                      # solve before factor
    x = torch.ones(n, dtype=torch.float64, device=dev)
    xbad = x.clone()
    xbad[5] = -1.0
    P.factor(xbad, x, 0.0, 0.0)
    with pytest.raises(ahlp.AHLPError) as e:
        P.solve(zn, zm, zn, max_refine=1)
    assert e.value.code == -5                      # x <= 0 seen by the factorization
    bad = gen.generate("tiny", 0)
    bad.A[2] = bad.A[2].copy()
    bad.A[2][0, 0] = np.nan
    with pytest.raises(ahlp.AHLPError) as e:
        ahlp.Problem(bad)
    assert e.value.code == -5
    bad = gen.generate("tiny", 0)
    bad.m = bad.m.copy()
    bad.m[1] = 100                                 # m > n
    with pytest.raises(ahlp.AHLPError) as e:
        ahlp.Problem(bad)
    assert e.value.code == -1
    _, _, _, res = P.ipm(max_iter=2)
    assert res["status"] == 1 and res["iterations"] == 2
    P.close()


def test_pivot_rule_counts_empty_row(dev):
    from paper_2412_07731_amd.ahlp import Problem
    inst = shaped(N=3, m=6, n=12, l=2, n0=2, seed=11)
    inst.A[1] = inst.A[1].copy()
    inst.A[1][2, :] = 0.0
    inst.C[1] = inst.C[1].copy()
    inst.C[1][2, :] = 0.0
    x, z, (rx, ry, rz) = point(inst, seed=8)
    ry[inst.yoff()[1] + 2] = 0.0
    P = Problem(inst)
    P.factor(T(x, dev), T(z, dev), 0.0, 0.0)
    dx, dy, dz, _ = P.solve(T(rx, dev), T(ry, dev), T(rz, dev))
    assert P.pivots() == 1
    f = newton.factor(inst, x, z, 0.0, 0.0)
    d = newton.solve(f, rx, ry, rz)
    for a, b in zip((dx, dy, dz), d):
        assert rel(H(a), b) < 1e-10
    P.close()


# ------------------------------------------------------------ full size
@pytest.fixture(scope="module")
def n512():
    return gen.generate("n512", 0)


def test_n512_direction_sampled(dev, n512):
    """N=512 (256 x 512 blocks, 16 links, 32 linking variables): the whole
    direction at a random point against the oracle, plus sampled block factors."""
    from paper_2412_07731_amd.ahlp import Problem
    inst = n512
    x, z, r = point(inst, seed=3)
    P = Problem(inst)
    P.factor(T(x, dev), T(z, dev), 1e-8, 1e-6)
    d = P.solve(*(T(v, dev) for v in r))
    f = newton.factor(inst, x, z, 1e-8, 1e-6)
    od = newton.solve(f, *r)
    for a, b in zip(d[:3], od):
        assert rel(H(a), b) < 1e-10
    for i in (0, 257, 511):
        Lg, Wg = P.debug_block(i)
        assert rel(Lg, f.L[i]) < 1e-12
        assert rel(Wg, f.W[i]) < 1e-11
    assert P.pivots() == 0          # also raises if the factorization reported an error
    P.close()


def test_n512_ipm_fp64(dev, n512):
    from paper_2412_07731_amd.ahlp import Problem
    g = golden("n512", 0)
    P = Problem(n512)
    x, y, z, res = P.ipm()
    print("n512 fp64", res["iterations"], res["primal_obj"], g["iterations"], g["pobj"], flush=True)
    assert res["status"] == 0
    assert res["iterations"] == g["iterations"]
    assert abs(res["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
    assert res["pivots_modified"] == 0
    check_trajectory(P.history(), res, g, "n512 fp64")
    P.close()


def test_n512_ipm_fp32_refine(dev, n512):
    """FP32 MFMA blocks with FP64 refinement reach the FP64 oracle's objective
    to 1e-8 (relative)."""
    from paper_2412_07731_amd.ahlp import Problem, FP32_REFINE
    g = golden("n512", 0)
    P = Problem(n512)
    x, y, z, res = P.ipm(precision=FP32_REFINE)
    err = abs(res["primal_obj"] - g["pobj"]) / max(1.0, abs(g["pobj"]))
    print("n512 fp32", res["iterations"], res["fp32_iterations"], err, res["refine_steps"], flush=True)
    assert res["status"] == 0
    assert res["fp32_iterations"] > 0
    assert err <= 1e-8
    P.close()


def _fp32_factor_bounds(A, D, L, W, B, delta):
    """Backward errors of FP32 block factors against the exact FP64 data
    (u = 2^-24).  The SYRK forms each M_ij as an n-term FP32 dot product
    (error <= (n + 2) u (|A| D |A'|)_ij, counting the rounding of A and D to
    FP32); the blocked Cholesky and the solve against B multiply by computed
    inverses of 16 x 16 diagonal tiles, whose own error adds a term
    ~ kappa_tile^2 u |L| |L'| (kappa_tile: the largest condition number of a
    diagonal tile of L).  Hence, component by component,
        |L L' - M| <= u ((n + 2) |A| D |A'| + (m + 1 + 4 kappa^2) |L| |L'|)
        |L W - B|  <= u ((m + 1 + 4 kappa^2) |L| |W| + |B|)
    (Higham, Accuracy and Stability, Thms 8.5 and 10.3, with the inverse
    terms of Sec. 14)."""
    u = 2.0 ** -24
    m, n = A.shape
    kap = 1.0
    for c in range(0, m, 16):
        Lt = L[c:c + 16, c:c + 16]
        kap = max(kap, np.linalg.cond(Lt, np.inf))
    M = (A * D) @ A.T + delta * np.eye(m)
    absM = (np.abs(A) * D) @ np.abs(A).T
    lhs_l = np.abs(L @ L.T - M)
    rhs_l = u * ((n + 2) * absM + (m + 1 + 4 * kap ** 2) * (np.abs(L) @ np.abs(L).T))
    lhs_w = np.abs(L @ W - B)
    rhs_w = u * ((m + 1 + 4 * kap ** 2) * (np.abs(L) @ np.abs(W)) + np.abs(B))
    return lhs_l, rhs_l, lhs_w, rhs_w, kap


# ragged blocks of 70-150 rows (5-10 tile rows, odd counts among them) with
# 4-20 link rows per pair: one-column last panels and waves with fewer rows
# than the panel kernel's maximum, in the FP32 panel factor's pipelined update
RAGGED_FP32 = dict(N=6, m=(70, 150), n="2m", l=(4, 20), n0=5, density=0.3)


@pytest.mark.parametrize("config", ["tiny", "n512", RAGGED_FP32], ids=["tiny", "n512", "ragged"])
def test_fp32_stage_parity(dev, config):
    """FP32 block factors (SYRK, Cholesky and W_i = L_i^-1 B_i in FP32 MFMA)
    against the FP64 oracle's blocks: the componentwise backward-error bounds
    of _fp32_factor_bounds hold, and the forward differences (printed) are of
    the order of kappa(M_i) u."""
    from paper_2412_07731_amd.ahlp import FP32_REFINE, Problem
    inst = gen.generate(config, 0)
    print("case fp32 stages", config, flush=True)
    x, z, _ = point(inst, seed=2)
    P = Problem(inst)
    try:
        P.factor(T(x, dev), T(z, dev), 1e-8, 1e-6, precision=FP32_REFINE)
        xo = inst.xoff()
        for i in sorted({0, 1, inst.N // 2, inst.N - 1}):
            Lg, Wg = P.debug_block(i)
            A = inst.A[i]
            D = 1.0 / (z[xo[i]:xo[i + 1]] / x[xo[i]:xo[i + 1]] + 1e-8)
            left, right = newton.link_cols(inst, i)
            B = np.hstack([(A * D) @ left.T, (A * D) @ right.T, inst.C[i]])
            ll, rl, lw, rw, kap = _fp32_factor_bounds(A, D, Lg, Wg, B, 1e-6)
            Lo = np.linalg.cholesky((A * D) @ A.T + 1e-6 * np.eye(A.shape[0]))
            print(f"  block {i}: |LL'-M| / bound {float(np.max(ll / np.maximum(rl, 1e-300))):.2e}, "
                  f"|LW-B| / bound {float(np.max(lw / np.maximum(rw, 1e-300))):.2e}, "
                  f"kappa_tile {kap:.1f}, forward L {rel(Lg, Lo):.1e}", flush=True)
            assert np.all(ll <= rl), ("L", i)
            assert np.all(lw <= rw), ("W", i)
    finally:
        P.close()
