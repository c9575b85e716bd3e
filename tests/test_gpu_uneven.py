"""GPU parity on uneven blocks (m_i ~ U{64..512}, n_i = 2 m_i, l_j ~ U{4..32},
64 linking variables):

* batched launches (blocks sorted largest first, block factor in two
  buckets on two streams) against one launch per block and stage: the
  interior-point runs must agree bit for bit;
* the N=2048 workload against the FP64 oracle (tests/golden): identical
  iteration count, objective within 1e-8; FP32+refine objective within 1e-8.
"""
import numpy as np
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


def test_batched_equals_per_block(dev):
    from paper_2412_07731_amd.ahlp import Problem
    print("case: uneven N=48 seed 1", flush=True)
    inst = gen.generate("uneven", 1, N=48)
    # bordered tile rows per block: m_i plus both link pairs and x_0, in tiles
    k = [(int(inst.l[j - 1]) if j > 0 else 0) + (int(inst.l[j]) if j < inst.N - 1 else 0) + inst.n0
         for j in range(inst.N)]
    rt = [(int(m) + 15) // 16 + (kk + 15) // 16 for m, kk in zip(inst.m, k)]
    assert max(rt) > 24 and min(rt) <= 24          # both factor buckets are used
    P = Problem(inst)
    try:
        x1, y1, z1, r1 = P.ipm()
        P.set_launch(per_block=True)
        x2, y2, z2, r2 = P.ipm()
        P.set_launch(per_block=False)
        assert r1["status"] == 0 and r2["status"] == 0
        assert r1["iterations"] == r2["iterations"]
        assert torch.equal(x1, x2) and torch.equal(y1, y2) and torch.equal(z1, z2)
        assert abs(r1["primal_obj"] - inst.fstar) <= 1e-7 * max(1.0, abs(inst.fstar))
    finally:
        P.close()


def test_uneven_full_size_against_oracle(dev):
    from paper_2412_07731_amd.ahlp import FP32_REFINE, Problem
    g = golden("uneven", 0)
    if g is None:
        pytest.skip("no oracle result for the uneven workload in tests/golden")
    print("case: uneven N=2048 seed 0", flush=True)
    inst = gen.generate("uneven", 0)
    P = Problem(inst)
    try:
        x, y, z, r = P.ipm()
        assert r["status"] == 0
        assert r["iterations"] == g["iterations"]
        assert abs(r["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
        check_trajectory(P.history(), r, g, "uneven fp64")
        x, y, z, r = P.ipm(precision=FP32_REFINE)
        assert r["status"] == 0
        assert abs(r["primal_obj"] - g["pobj"]) <= 1e-8 * max(1.0, abs(g["pobj"]))
    finally:
        P.close()


def test_autotune_table(dev, tmp_path):
    from paper_2412_07731_amd.ahlp import Problem
    print("case: autotune uneven N=48 seed 1", flush=True)
    inst = gen.generate("uneven", 1, N=48)
    path = str(tmp_path / "tune.txt")
    P = Problem(inst)
    try:
        n = P.autotune(path)
        rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
        assert n >= 1 and len(rows) == n
        kinds = set()
        for arch, rt, kern, us_p, us_c, us_p8 in rows:
            assert 1 <= int(rt) <= 40
            t = {"panel": float(us_p), "column": float(us_c), "panel8": float(us_p8)}
            t = {k: v for k, v in t.items() if v >= 0}          # -1: the kernel cannot hold them
            assert t[kern] == min(t.values()), (rt, kern, t)
            assert (int(rt) <= 24) == ("panel" in t)
            kinds.add(kern)
        print("autotuned kernels:", sorted(kinds), flush=True)
        x, y, z, r = P.ipm()
        assert r["status"] == 0
        assert abs(r["primal_obj"] - inst.fstar) <= 1e-7 * max(1.0, abs(inst.fstar))
    finally:
        P.close()
    P2 = Problem(inst)
    try:
        assert P2.autotune(path) == 0          # every entry from the cache
    finally:
        P2.close()


@pytest.mark.parametrize("case", ["tiny", "uneven48", "n512"])
def test_launch_modes_bitwise(dev, case):
    """One launch per stage (the default), one launch per block and stage, and
    the fused persistent launch (link columns, SYRK, block factor and Schur
    contributions of the panel bucket) give bitwise the same factors and
    Newton direction."""
    from paper_2412_07731_amd.ahlp import Problem
    print("case: launch modes", case, flush=True)
    inst = gen.generate("uneven", 1, N=48) if case == "uneven48" else gen.generate(case, 0)
    rng = np.random.default_rng(4)
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    x, z = T(rng.uniform(0.1, 2, inst.n_tot)), T(rng.uniform(0.1, 2, inst.n_tot))
    r = (T(rng.standard_normal(inst.n_tot)), T(rng.standard_normal(inst.m_tot)),
         T(rng.standard_normal(inst.n_tot)))
    blocks = sorted({0, 1, inst.N // 3, inst.N // 2, inst.N - 1})
    P = Problem(inst)
    try:
        out = {}
        for mode in ("batched", "fused", "per_block"):
            P.set_launch(mode=mode)
            P.factor(x, z, 1e-8, 1e-6)
            d = P.solve(*r, max_refine=2)
            torch.cuda.synchronize()
            out[mode] = ([P.debug_block(i) for i in blocks], d)
        P.set_launch(mode="batched")
        ref_blocks, ref_d = out["batched"]
        for mode in ("fused", "per_block"):
            bl, d = out[mode]
            for (L1, W1), (L2, W2) in zip(ref_blocks, bl):
                assert np.array_equal(L1, L2) and np.array_equal(W1, W2), (case, mode)
            assert all(torch.equal(a, b) for a, b in zip(ref_d[:3], d[:3])), (case, mode)
    finally:
        P.close()
