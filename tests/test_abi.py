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


STRUCTS = [("ahlp_problem_desc_t", "Desc"), ("ahlp_factor_opts_t", "FactorOpts"),
           ("ahlp_ipm_opts_t", "IpmOpts"), ("ahlp_ipm_result_t", "IpmResult"),
           ("ahlp_ipm_iter_t", "IpmIter")]


def test_struct_layouts(tmp_path):
    """Every binding structure has the size and field offsets that the C
    compiler gives the header's declaration."""
    from paper_2412_07731_amd import ahlp
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ahlp.h"', "int main(void) {"]
    for cname, pyname in STRUCTS:
        lines.append(f'  printf("{pyname} size %zu\\n", sizeof({cname}));')
        for f, _ in getattr(ahlp, pyname)._fields_:
            lines.append(f'  printf("{pyname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("no C compiler or HIP headers")
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        pyname, field, val = line.split()
        S = getattr(ahlp, pyname)
        got = ctypes.sizeof(S) if field == "size" else getattr(S, field).offset
        assert got == int(val), (pyname, field, got, val)


def test_library_fails_loudly_when_missing(monkeypatch, tmp_path):
    from paper_2412_07731_amd import ahlp
    monkeypatch.setattr(ahlp, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(ahlp, "_lib", None)
    with pytest.raises(RuntimeError):
        ahlp.lib()
