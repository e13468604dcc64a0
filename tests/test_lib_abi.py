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
    assert ctypes.sizeof(P) == 48 + 8 * 19
    assert ctypes.sizeof(mps.StepStats) == 56


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2105_01677_amd import mps, workloads as W
    w = W.config("cfg1")
    with pytest.raises(RuntimeError):
        mps.MPS(w.params, w.pos, w.vel, w.ptype)
