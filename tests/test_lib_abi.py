"""Host-side checks of the C ABI: the HIP library builds, loads without a
GPU, and exports every function that include/mps.h declares; the ctypes
mirror of mps_params matches the C layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mps_init", "mps_neighbors", "mps_step", "mps_pressure_solve"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2105_01677_amd import mps
    if not os.path.exists(mps.LIB_PATH):
        from paper_2105_01677_amd import build
        build.build()
    lib = ctypes.CDLL(mps.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(mps.EXPORTED) == set(declared_functions())


def test_params_layout():
    from paper_2105_01677_amd import mps
    P = mps.Params
    assert P.l0.offset == 48          # 12 int32 before the doubles
    assert P.source.offset == 48 + 8 * 19      # then int32 laplacian, double skin
    assert P.laplacian.offset == P.source.offset + 4
    assert P.skin.offset == 48 + 8 * 20
    assert P.precond.offset == 48 + 8 * 21
    assert ctypes.sizeof(P) == 48 + 8 * 22
    assert ctypes.sizeof(mps.StepStats) == 72
    assert mps.StepStats.cg_redone.offset == 56
    assert mps.StepStats.list_builds.offset == 60
    assert mps.StepStats.short_entries.offset == 64


def test_struct_layouts_match_the_c_header(tmp_path):
    """The ctypes mirrors against the header compiled by the host C
    compiler: sizes and every field offset."""
    import shutil
    import subprocess
    from paper_2105_01677_amd import mps
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mps.h"', "int main(void) {"]
    for cname, py in (("mps_params", mps.Params), ("mps_step_stats", mps.StepStats)):
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, f, v = line.split()
        got[(cname, f)] = int(v)
    for cname, py in (("mps_params", mps.Params), ("mps_step_stats", mps.StepStats)):
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2105_01677_amd import mps, workloads as W
    w = W.config("dam_break_2d_1432")
    with pytest.raises(RuntimeError):
        mps.MPS(w.params, w.pos, w.vel, w.ptype)
