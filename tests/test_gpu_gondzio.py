"""GPU parity with Gondzio's multiple centrality correctors (opts.gondzio = 2):
identical iteration counts and kept-corrector counts (per iteration), the
per-iterate backward-error and mu parity of the runs without correctors,
objective within 1e-8 of
the FP64 oracle with the same correctors (tests/golden), on the tiny workload
(seeds 0-7) and N=512; FP32+refine with correctors reaches the same objective."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2412_07731_amd import gen  # noqa: E402
from tests._parity import check_trajectory, golden  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_07731_amd import ahlp
    ahlp.lib()          # raises if the library is missing: no silent fallback
    return torch.device("cuda", 0)


@pytest.mark.parametrize("config,seed", [("tiny", s) for s in range(8)] + [("n512", 0)])
def test_gondzio_parity(dev, config, seed):
    from paper_2412_07731_amd.ahlp import FP32_REFINE, Problem
    g = golden(config, seed, 2)
    if g is None:
        pytest.skip("no oracle result with correctors in tests/golden")
    print("case:", config, seed, flush=True)
    P = Problem(gen.generate(config, seed))
    try:
        x, y, z, r = P.ipm(gondzio=2)
        assert r["status"] == 0
        assert r["iterations"] == g["iterations"]
        assert r["correctors"] == g["correctors"]
        assert abs(r["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
        hist = P.history()
        assert [h["correctors"] for h in hist] == g["correctors_trace"]
        check_trajectory(hist, r, g, f"{config} seed {seed} gondzio 2")
        if config == "tiny":
            x, y, z, r = P.ipm(gondzio=2, precision=FP32_REFINE)
            assert r["status"] == 0
            assert abs(r["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
    finally:
        P.close()
