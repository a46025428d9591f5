"""CPU-side checks of the C ABI: the built library loads and exports every
symbol the public header declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "mgfr.h")
LIB = os.path.join(ROOT, "paper_1305_2418_amd", "libmgfr.so")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"\b(mgfr_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("mgfr_assign_density", "mgfr_solve", "mgfr_fifth_force", "mgfr_create",
              "mgfr_destroy", "mgfr_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgfr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmgfr.so not built")
def test_host_only_calls_work_without_gpu():
    from paper_1305_2418_amd import mgfr
    fb, beta, C = mgfr.background(mgfr.Params(a=0.5, fr0_abs=1e-6))
    assert fb == pytest.approx(1e-6 * ((1 + 4 * 0.7 / 0.3) / (8 + 4 * 0.7 / 0.3)) ** 2)
    with pytest.raises(mgfr.MgfrError):
        mgfr.background(mgfr.Params(mesh=24))
    assert mgfr.exported_symbols() == declared()
