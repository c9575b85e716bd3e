"""The C-ABI library loads and exports every function include/ahlp.h declares,
and the binding's structures match the header's sizes (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ahlp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ahlp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["ahlp_problem_create", "ahlp_problem_destroy", "ahlp_kkt_factor",
                     "ahlp_kkt_solve", "ahlp_ipm_solve", "ahlp_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2412_07731_amd import ahlp
    if not os.path.exists(ahlp.LIB_PATH):
        pytest.skip("libahlp.so not built")
    L = ctypes.CDLL(ahlp.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    # the binding knows every declared function
    assert set(declared_functions()) == set(ahlp.SIGNATURES)


def test_struct_layouts():
    from paper_2412_07731_amd import ahlp
    # 2 int32 + 3 pointers + 7 pointers
    assert ctypes.sizeof(ahlp.Desc) == 8 + 10 * 8
    assert ctypes.sizeof(ahlp.FactorOpts) == 24
    assert ctypes.sizeof(ahlp.IpmResult) == 5 * 4 + 4 + 8 * 8 + 8 * 8 + 8 * 4 + 8 + 8


def test_library_fails_loudly_when_missing(monkeypatch, tmp_path):
    from paper_2412_07731_amd import ahlp
    monkeypatch.setattr(ahlp, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(ahlp, "_lib", None)
    with pytest.raises(RuntimeError):
        ahlp.lib()
