"""Graph mode of the interior-point driver (opts.graph = 1): each iteration's
factorization is captured once as a hipGraph and replayed.  The replays run
between the iterations' own eager kernels and host synchronizations; since the
graph holds the same kernels with the same arguments, every run must equal the
eager run bit for bit (a wrong replay would change the iterates).  Cases: the
tiny workload in FP64 and FP32+refine, uneven blocks (both factor buckets, so
the two-stream fork is inside the capture), and the N=512 workload; each graph
run is done twice so the second reuses the cached graph."""
import time

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


def _same(a, b):
    return all(torch.equal(u, v) for u, v in zip(a[:3], b[:3])) and a[3]["iterations"] == b[3]["iterations"]


@pytest.mark.parametrize("case", ["tiny", "uneven48", "n512"])
def test_graph_equals_eager(dev, case):
    from paper_2412_07731_amd.ahlp import FP32_REFINE, FP64, Problem
    print("case:", case, flush=True)
    inst = gen.generate("uneven", 1, N=48) if case == "uneven48" else gen.generate(case, 0)
    P = Problem(inst)
    try:
        precs = [FP64, FP32_REFINE] if case == "tiny" else [FP64]
        for prec in precs:
            torch.cuda.synchronize()
            t = time.perf_counter()
            e = P.ipm(precision=prec)
            torch.cuda.synchronize()
            te = time.perf_counter() - t
            assert e[3]["status"] == 0
            for rep in range(2):
                torch.cuda.synchronize()
                t = time.perf_counter()
                g = P.ipm(precision=prec, graph=1)
                torch.cuda.synchronize()
                tg = time.perf_counter() - t
                assert _same(e, g), (case, prec, rep)
            print(f"{case} prec {prec}: eager {1e3 * te:.1f} ms, graph {1e3 * tg:.1f} ms", flush=True)
    finally:
        P.close()
