"""ahlp_kkt_solve_noalloc (the solve with its workspace in the library's
static device array, for callers that cannot allocate) against
ahlp_kkt_solve on the same factors and right-hand sides, through the C ABI:
bit-identical directions and backward errors, on two calls in a row (the
N=512 workload, then the smaller tiny one, which must not see the first
call's leftovers), with and without refinement; the handle's own solve still
works afterwards; a problem whose workspace exceeds the array is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2412_07731_amd import gen  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_07731_amd import ahlp
    ahlp.lib()          # raises if the library is missing: no silent fallback
    return torch.device("cuda", 0)


def _case(inst, dev, seed):
    rng = np.random.default_rng(seed)
    n, m = inst.n_tot, inst.m_tot
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    x, z = T(rng.uniform(0.1, 2, n)), T(rng.uniform(0.1, 2, n))
    r = (T(rng.standard_normal(n)), T(rng.standard_normal(m)), T(rng.standard_normal(n)))
    return x, z, r


def _same(a, b):
    return all(torch.equal(u, v) for u, v in zip(a[:3], b[:3])) and a[3] == b[3]


def test_noalloc_matches_solve_two_calls(dev):
    from paper_2412_07731_amd.ahlp import Problem
    for config, seed in (("n512", 0), ("tiny", 1)):      # the second call is smaller
        print("case: noalloc", config, flush=True)
        inst = gen.generate(config, seed)
        P = Problem(inst)
        try:
            x, z, r = _case(inst, dev, seed + 7)
            P.factor(x, z, 1e-8, 1e-6)
            for refine in (5, 0):
                ref = P.solve(*r, max_refine=refine, refine_tol=1e-10)
                got = P.solve_noalloc(*r, max_refine=refine, refine_tol=1e-10)
                torch.cuda.synchronize()
                assert _same(ref, got), (config, refine)
            again = P.solve(*r, max_refine=5, refine_tol=1e-10)   # the handle's workspace is back
            assert _same(again, P.solve(*r, max_refine=5, refine_tol=1e-10))
        finally:
            P.close()


def test_noalloc_refuses_oversized_problem(dev):
    from paper_2412_07731_amd.ahlp import AHLPError, Problem
    print("case: noalloc oversized", flush=True)
    inst = gen.generate(dict(N=1024, m=16, n=1024, l=2, n0=0, density=0.02), 0)
    P = Problem(inst)
    try:
        x, z, r = _case(inst, dev, 3)
        P.factor(x, z, 1e-8, 1e-6)
        with pytest.raises(AHLPError) as e:
            P.solve_noalloc(*r)
        assert e.value.code == -1 and "static workspace" in str(e.value)
    finally:
        P.close()
