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
    # a batch wider than the widest interleaved cycle (32 columns)
    bad = fracprec.default_options(max_batch=33)
    assert lib.fpc_create(ctypes.byref(h), ctypes.byref(bad), None) == -1
    assert not h.value
    # calls on a null handle fail cleanly
    assert lib.fpc_apply_prec(None, None, None) == -1
    assert lib.fpc_num_levels(None) == 0


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the sizes and field offsets
    the C compiler gives the header's definitions."""
    import shutil
    import subprocess
    from paper_2112_12397_amd import fracprec as F
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"fpc_csr": F.FpcCsr, "fpc_block_system": F.FpcBlockSystem,
               "fpc_amg_options": F.FpcAmgOptions, "fpc_options": F.FpcOptions,
               "fpc_info": F.FpcInfo, "fpc_level_desc": F.FpcLevelDesc,
               "fpc_flow_graph": F.FpcFlowGraph,
               "fpc_pressure_desc": F.FpcPressureDesc}
    lines = ['#include <stdio.h>', '#include <stddef.h>',
             '#include "fracprec.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", '
                         f'offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            parts = line.split()
            got[tuple(parts[:-1])] = int(parts[-1])
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, \
                (cname, fname)
