"""The device-ceiling measurement aids (ahlp_ceiling_mfma, ahlp_ceiling_hbm_read,
ahlp_ceiling_tile_chol): positive rates no higher than the device can deliver
(the published MI355X figures with 5% slack for clock variation), a tile
Cholesky latency within the bounds its instruction count allows, and refusal
of bad arguments."""
import pytest

torch = pytest.importorskip("torch")

from paper_2412_07731_amd import ahlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def test_mfma_ceilings(dev):
    print("case: mfma ceilings", flush=True)
    f64 = ahlp.ceiling_mfma(ahlp.FP64)
    f32 = ahlp.ceiling_mfma(ahlp.FP32_REFINE)
    print(f"  FP64 {f64:.1f} TFLOP/s, FP32 {f32:.1f} TFLOP/s", flush=True)
    assert 0.0 < f64 <= 1.05 * 78.6
    assert 0.0 < f32 <= 1.05 * 157.3
    assert ahlp.lib().ahlp_ceiling_mfma(ahlp.FP64, None, None) == -1          # null output
    assert ahlp.lib().ahlp_ceiling_mfma(7, ahlp.C.byref(ahlp.C.c_double()), None) == -1


def test_hbm_read_ceiling(dev):
    print("case: hbm read ceiling, 1 GiB", flush=True)
    buf = torch.zeros(1 << 27, dtype=torch.float64, device=dev)
    g = ahlp.ceiling_hbm_read(buf)
    print(f"  {g:.0f} GB/s", flush=True)
    assert 0.0 < g <= 1.05 * 8000.0
    assert buf.abs().sum().item() == 0.0   # read, never written
    v = ahlp.C.c_double()
    assert ahlp.lib().ahlp_ceiling_hbm_read(None, 1 << 20, ahlp.C.byref(v), None) == -1
    assert ahlp.lib().ahlp_ceiling_hbm_read(ahlp._dptr(buf), 1, ahlp.C.byref(v), None) == -1


def test_tile_chol_latency(dev):
    print("case: tile Cholesky latency, alone and beside an MFMA stream", flush=True)
    alone = ahlp.ceiling_tile_chol(False)
    beside = ahlp.ceiling_tile_chol(True)
    print(f"  alone {alone:.2f} us, beside FP64 MFMAs {beside:.2f} us", flush=True)
    # 16 dependent elimination steps of at least ~40 instructions issue in no
    # less than 16*40*4 cycles (0.1 us at 2.4 GHz); far more than 50 us would
    # mean the loop is not what is timed
    assert 0.1 < alone < 50.0
    assert 0.1 < beside < 50.0
    v = ahlp.C.c_double()
    assert ahlp.lib().ahlp_ceiling_tile_chol(0, None, None) == -1
    assert ahlp.lib().ahlp_ceiling_tile_chol(2, ahlp.C.byref(v), None) == -1
