"""The C-ABI library loads and exports every entry point the header declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fracprec.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpc_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("fpc_setup", "fpc_apply_prec", "fpc_solve", "fpc_solve_T",
              "fpc_solve_batch", "fpc_grad_log_trans"):
        assert n in names


def test_library_exports_every_symbol():
    from paper_2112_12397_amd import fracprec
    if not os.path.exists(fracprec.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fracprec.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(fracprec.EXPORTS)
    fracprec.load_library()


def test_default_options_and_status_strings():
    from paper_2112_12397_amd import fracprec
    if not os.path.exists(fracprec.LIB_PATH):
        pytest.skip("library not built")
    lib = fracprec.load_library()
    o = fracprec.default_options()
    assert o.restart == 50 and o.rtol == 1e-8 and o.amg.max_coarse == 2000
    assert o.amg.cheb_degree == 2 and abs(o.amg.omega_factor - 4 / 3) < 1e-15
    for st in fracprec.STATUS:
        assert lib.fpc_status_string(st)
    # invalid options are rejected without touching a device
    h = ctypes.c_void_p()
    bad = fracprec.default_options(restart=0)
    assert lib.fpc_create(ctypes.byref(h), ctypes.byref(bad), None) == -1
    # calls on a null handle fail cleanly
    assert lib.fpc_apply_prec(None, None, None) == -1
    assert lib.fpc_num_levels(None) == 0
