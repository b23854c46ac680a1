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


@pytest.mark.skipif(not os.path.exists(rst.LIB_PATH), reason="librst.so not built")
def test_host_side_argument_errors_and_defaults():
    """Documented behaviour that needs no device: null contexts and outputs are
    refused with RST_EINVAL before any HIP call, rst_destroy(NULL) is a no-op,
    the network's weight count follows the documented layer layout and the
    low-rank options have their documented defaults."""
    lib = rst.load()
    assert lib.rst_create(None, 0, None) == rst.RST_EINVAL
    lib.rst_destroy(None)
    assert lib.rst_last_error(None) == b"null context"
    assert lib.rst_set_grid(None, 8, 8, 8, 0.5, 0.5, 0.5, 4) == rst.RST_EINVAL
    assert lib.rst_set_k(None, 0.0, 0.0) == rst.RST_EINVAL
    assert lib.rst_set_solver(None, None) == rst.RST_EINVAL
    d = ctypes.c_double()
    assert lib.rst_apply_timing(None, ctypes.byref(d), ctypes.byref(d)) == rst.RST_EINVAL
    # layers W0..W8: (cout, cin) = (16, 4), (16, 16) x 7, (2, 16), 27 taps each
    assert lib.rst_cnn_weight_count() == 27 * (16 * 4 + 7 * 16 * 16 + 2 * 16)
    o = rst.rst_lowrank_opts()
    lib.rst_default_lowrank(ctypes.byref(o))
    assert (o.probes, o.heldout, o.max_probes, o.tail_tol) == (32, 8, 256, 1e-7)
    lib.rst_default_lowrank(None)  # ignored
