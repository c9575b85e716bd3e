"""GPU parity of the general form (bounds and inequality rows, Sec. 3.2)
through paper_2412_07731_amd.general, against the oracle's own
reformulation and IPM (tests/golden, written by make_golden.py):

* the same iteration count, objective within 1e-8 relative, the recovered x
  feasible in the general form within 1e-7 (g_small seeds 0-3: 6 blocks with
  every bound and row kind; g_medium: 64 blocks of 48..96 equality and 8..24
  inequality rows, 8 linking variables; g_large: 256 blocks of 96..160
  equality and 16..48 inequality rows, 16 linking variables);
* FP32+refine on g_medium: objective within 1e-8.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2412_07731_amd import gen  # noqa: E402

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_ipm.json")))


def golden(config, seed):
    for r in GOLDEN["runs"]:
        if r["config"] == config and r["seed"] == seed and not r.get("dense") and not r.get("bounds"):
            return r
    raise KeyError((config, seed))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_07731_amd import ahlp
    ahlp.lib()          # raises if the library is missing: no silent fallback
    return torch.device("cuda", 0)


def violation(g, x):
    Aeq, beq, Ain, dv, fv = gen.general_matrices(g)
    r = Ain @ x
    return max(float(np.max(np.abs(Aeq @ x - beq), initial=0.0)),
               float(np.max(np.maximum(dv - r, 0.0), initial=0.0)),
               float(np.max(np.maximum(r - fv, 0.0), initial=0.0)),
               float(np.max(np.maximum(g.lo - x, 0.0))), float(np.max(np.maximum(x - g.up, 0.0))))


@pytest.mark.parametrize("config,seed", [("g_small", 0), ("g_small", 1), ("g_small", 2),
                                         ("g_small", 3), ("g_medium", 0), ("g_large", 0)])
def test_general_against_oracle(dev, config, seed):
    from paper_2412_07731_amd import general
    print("case: general", config, seed, flush=True)
    g = gen.generate_general(config, seed)
    ref = golden(config, seed)
    x, f, res = general.solve(g)
    assert res["status"] == 0
    assert res["iterations"] == ref["iterations"]
    assert abs(f - ref["objective"]) <= 1e-8 * max(1.0, abs(ref["objective"]))
    assert violation(g, x) <= 1e-7


def test_general_fp32_refine(dev):
    from paper_2412_07731_amd import general
    from paper_2412_07731_amd.ahlp import FP32_REFINE
    print("case: general g_medium 0 fp32", flush=True)
    g = gen.generate_general("g_medium", 0)
    ref = golden("g_medium", 0)
    x, f, res = general.solve(g, precision=FP32_REFINE)
    assert res["status"] == 0
    assert abs(f - ref["objective"]) <= 1e-8 * max(1.0, abs(ref["objective"]))
    assert violation(g, x) <= 1e-7
