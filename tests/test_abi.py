"""The C-ABI library loads and exports every symbol include/rst.h declares (CPU)."""
import ctypes
import os
import re

import pytest

from paper_2208_02783_amd import rst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "rst.h")).read()
    return sorted(set(re.findall(r"\b(rst_[a-z_0-9]+)\s*\(", txt)))


def test_header_lists_the_binding_names():
    assert set(header_symbols()) == set(rst.EXPORTED)


@pytest.mark.skipif(not os.path.exists(rst.LIB_PATH), reason="librst.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rst.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(rst.LIB_PATH), reason="librst.so not built")
def test_default_solver_options():
    o = rst.default_solver()
    assert o.tol == 1e-10 and o.max_iter > 0 and o.method == rst.RST_BICGSTAB
    assert o.direction == rst.RST_DIR_LR


def test_missing_library_fails_loudly(tmp_path):
    saved = rst._lib
    rst._lib = None
    try:
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            rst.load(str(tmp_path / "nope.so"))
    finally:
        rst._lib = saved
