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


def test_graph_recaptured_after_autotune(dev, tmp_path):
    """A captured iteration holds the block-factor buckets and their launch
    geometry.  Autotuning (which can move blocks between the panel and the
    column kernel) and a change of launch mode must make the next graph run
    capture again: every graph run equals the eager run of the same
    configuration bit for bit."""
    from paper_2412_07731_amd.ahlp import Problem
    print("case: uneven48 graph + autotune + launch mode", flush=True)
    inst = gen.generate("uneven", 1, N=48)
    P = Problem(inst)
    try:
        e0 = P.ipm()
        assert _same(e0, P.ipm(graph=1))
        # a table that sends every tunable block to the column kernel
        path = tmp_path / "tune.txt"
        t16 = lambda v: (int(v) + 15) // 16  # noqa: E731
        # bordered tile rows of block j: its rows, then each link pair's and
        # x_0's columns, each rounded up to whole tiles
        rts = sorted({t16(inst.m[j]) + (t16(inst.l[j - 1]) if j > 0 else 0)
                      + (t16(inst.l[j]) if j < inst.N - 1 else 0) + t16(inst.n0)
                      for j in range(inst.N)})
        import torch as _t
        arch = _t.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        path.write_text("".join(f"{arch} {rt} column 1.0 0.5 1.0\n" for rt in rts if rt <= 40))
        assert P.autotune(str(path)) == 0
        e1 = P.ipm()
        g1 = P.ipm(graph=1)
        assert _same(e1, g1)
        P.set_launch(per_block=True)
        g2 = P.ipm(graph=1)
        P.set_launch(per_block=False)
        assert _same(e1, g2)
    finally:
        P.close()
