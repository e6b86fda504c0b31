"""Host-only checks of the C ABI: the library loads, exports every symbol the header
declares, and validates grids without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(lbfd_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary():
    names = header_symbols()
    for required in ("lbfd_create", "lbfd_set_params", "lbfd_set_walls", "lbfd_set_fields",
                     "lbfd_step", "lbfd_get_fields", "lbfd_diagnostics", "lbfd_destroy",
                     "lbfd_state_bytes", "lbfd_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1406_2686_amd as lb

    lib = lb.raw()
    missing = [n for n in header_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_state_bytes_validates_grid():
    import paper_1406_2686_amd as lb

    assert lb.state_bytes(16, 32, 16, 1) > 0
    b1 = lb.state_bytes(128, 64, 128, 2)
    # two population copies (2 x 19 FP32) and two C copies (6 FP32) at least
    assert b1 >= 128 * 64 * 128 * (2 * 2 * 19 + 2 * 6) * 4
    # ny >= 3, ncomp in {1, 2}, positive extents, fewer than 2^30 nodes
    for bad in [(16, 2, 16, 1), (0, 8, 8, 1), (8, 8, 8, 3), (8, 8, -1, 2), (1024, 1024, 1024, 1)]:
        with pytest.raises(lb.LbfdError):
            lb.state_bytes(*bad)


def test_structs_match_header_layout():
    import paper_1406_2686_amd as lb

    assert ctypes.sizeof(lb.Grid) == 16
    assert ctypes.sizeof(lb.Params) == 8 * 6 + 8 + 8 * 3 + 8 + 8
    assert ctypes.sizeof(lb.Diag) == 8 * (2 + 3 + 1 + 3 + 6 + 5) + 8 + 8 + 8


def test_struct_offsets_match_the_compiled_header(tmp_path):
    """Every field of the ctypes mirrors sits at the offset the C compiler gives it when
    compiling include/lbfd.h (the header needs only <stdint.h>)."""
    import shutil
    import subprocess

    import paper_1406_2686_amd as lb

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    pairs = [("lbfd_grid", lb.Grid), ("lbfd_params", lb.Params), ("lbfd_diag", lb.Diag),
             ("lbfd_tuning", lb.Tuning), ("lbfd_steady_crit", lb.SteadyCrit), ("lbfd_train_opts", lb.TrainOpts),
             ("lbfd_walls", lb.Walls)]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lbfd.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-I", inc, str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
