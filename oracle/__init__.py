"""MPS oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around the plain FP64 C++ reference in ``mps_oracle.cpp``.
Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the HIP library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmps_oracle.so")
SOURCES = ["mps_oracle.cpp"]


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (FP64, OpenMP, no FMA contraction so the
    squared-distance expression rounds term by term)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-o", LIB_PATH + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class OrcParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("pmode", C.c_int32), ("kernel", C.c_int32),
        ("grad", C.c_int32), ("clamp", C.c_int32), ("max_neigh", C.c_int32),
        ("cg_maxit", C.c_int32), ("grid_n", C.c_int32 * 3),
        ("l0", C.c_double), ("re_n", C.c_double), ("re_lap", C.c_double),
        ("rho", C.c_double), ("nu", C.c_double), ("g", C.c_double * 3),
        ("dt", C.c_double), ("beta", C.c_double), ("c0", C.c_double),
        ("gamma", C.c_double), ("alpha", C.c_double), ("cg_tol", C.c_double),
        ("grid_lo", C.c_double * 3), ("cell_size", C.c_double),
        ("smag_cs", C.c_double), ("source", C.c_int32), ("laplacian", C.c_int32),
        ("cg_warm", C.c_int32),
    ]


class OrcStepOut(C.Structure):
    _fields_ = [
        ("cell", C.c_void_p), ("count", C.c_void_p), ("list", C.c_void_p),
        ("us", C.c_void_p), ("rs", C.c_void_p), ("nstar", C.c_void_p),
        ("flags", C.c_void_p), ("diag", C.c_void_p), ("b", C.c_void_p),
        ("aval", C.c_void_p), ("p", C.c_void_p), ("phat", C.c_void_p),
        ("gradp", C.c_void_p), ("nut", C.c_void_p), ("pos", C.c_void_p), ("vel", C.c_void_p),
        ("type", C.c_void_p), ("cg_iters", C.c_int32), ("cg_relres", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_weight.restype = C.c_double
        L.orc_weight.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_lattice_constants.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int,
                                            C.POINTER(C.c_double), C.POINTER(C.c_double),
                                            C.POINTER(C.c_int32)]
        for f in (L.orc_neighbors_brute,):
            f.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                          C.c_void_p, C.c_void_p]
        L.orc_neighbors_cells.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(OrcStepOut)]
        L.orc_run.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p]
        L.orc_smoothed_density.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Host threads of the oracle's OpenMP loops; returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def make_params(p: dict) -> OrcParams:
    o = OrcParams()
    for k in ("dim", "pmode", "kernel", "grad", "clamp", "max_neigh", "cg_maxit"):
        setattr(o, k, int(p[k]))
    for k in ("l0", "re_n", "re_lap", "rho", "nu", "dt", "beta", "c0", "gamma",
              "alpha", "cg_tol", "cell_size", "smag_cs"):
        setattr(o, k, float(p[k]))
    o.source = int(p.get("source", 0))
    o.laplacian = int(p.get("laplacian", 0))
    o.cg_warm = int(p.get("cg_warm", 0))
    for a in range(3):
        o.g[a] = float(p["g"][a])
        o.grid_lo[a] = float(p["grid_lo"][a])
        o.grid_n[a] = int(p["grid_n"][a])
    return o


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def weight(kernel: int, r: float, re: float) -> float:
    return lib().orc_weight(kernel, r, re)


def lattice_constants(dim: int, l0: float, re: float, kernel: int):
    """(n0, lambda, neighbour count) of an interior lattice particle."""
    n0, lam, cnt = C.c_double(), C.c_double(), C.c_int32()
    lib().orc_lattice_constants(dim, l0, re, kernel, C.byref(n0), C.byref(lam), C.byref(cnt))
    return n0.value, lam.value, cnt.value


def _prep(params, pos, ptype):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    ptype = np.ascontiguousarray(ptype, dtype=np.int8)
    return make_params(params), pos, ptype


def neighbors_brute(params, pos, ptype):
    """(status, count[n], list[n][max_neigh]) by all-pairs search."""
    P, pos, ptype = _prep(params, pos, ptype)
    n = pos.shape[0]
    cnt = np.zeros(n, np.int32)
    lst = np.zeros((n, P.max_neigh), np.int32)
    st = lib().orc_neighbors_brute(C.byref(P), n, _ptr(pos), _ptr(ptype), _ptr(cnt), _ptr(lst))
    return st, cnt, lst


def neighbors_cells(params, pos, ptype):
    """(status, cell[n], count[n], list[n][max_neigh]) by the cell-linked list."""
    P, pos, ptype = _prep(params, pos, ptype)
    n = pos.shape[0]
    cell = np.zeros(n, np.int32)
    cnt = np.zeros(n, np.int32)
    lst = np.zeros((n, P.max_neigh), np.int32)
    st = lib().orc_neighbors_cells(C.byref(P), n, _ptr(pos), _ptr(ptype), _ptr(cell),
                                   _ptr(cnt), _ptr(lst))
    return st, cell, cnt, lst


def _opt(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def step(params, pos, vel, ptype, flags_override=None, *, want_lists=True,
         want_matrix=False, rho_s=None, nu_i=None):
    """One time step.  Returns (status, dict of fields)."""
    P, pos, ptype = _prep(params, pos, ptype)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    n, dim = pos.shape
    K = P.max_neigh
    out = {
        "cell": np.zeros(n, np.int32),
        "count": np.zeros(n, np.int32),
        "us": np.zeros((n, dim)), "rs": np.zeros((n, dim)),
        "nstar": np.zeros(n), "flags": np.zeros(n, np.int8),
        "diag": np.zeros(n), "b": np.zeros(n),
        "p": np.zeros(n), "phat": np.zeros(n), "gradp": np.zeros((n, dim)),
        "nut": np.zeros(n),
        "pos": np.zeros((n, dim)), "vel": np.zeros((n, dim)),
        "type": np.zeros(n, np.int8),
    }
    if want_lists:
        out["list"] = np.zeros((n, K), np.int32)
    if want_matrix:
        out["aval"] = np.zeros((n, K))
    so = OrcStepOut()
    for k, v in out.items():
        setattr(so, k, v.ctypes.data)
    fo = None
    if flags_override is not None:
        fo = np.ascontiguousarray(flags_override, dtype=np.int8)
    rs_, nu_ = _opt(rho_s), _opt(nu_i)
    st = lib().orc_step(C.byref(P), n, _ptr(pos), _ptr(vel), _ptr(ptype), _ptr(fo),
                        _ptr(rs_), _ptr(nu_), C.byref(so))
    out["cg_iters"] = so.cg_iters
    out["cg_relres"] = so.cg_relres
    return st, out


def run(params, pos, vel, ptype, nsteps, *, rho_s=None, nu_i=None, return_iters=False,
        p0=None):
    """nsteps time steps; returns (status, pos, vel, type, p, flags), plus the
    CG iterations summed over the steps when return_iters.  With
    params["cg_warm"] = 1 each solve starts from the previous step's pressure
    (p0 for the first step, if given) and stops at params["cg_tol"] (the GPU
    path's rule) instead of starting from zero and stopping at 1e-13."""
    P, pos, ptype = _prep(params, pos, ptype)
    pos = pos.copy()
    ptype = ptype.copy()
    vel = np.ascontiguousarray(vel, dtype=np.float64).copy()
    n = pos.shape[0]
    p = np.zeros(n) if p0 is None else np.array(p0, dtype=np.float64)
    fl = np.zeros(n, np.int8)
    it = C.c_int64(0)
    rs_, nu_ = _opt(rho_s), _opt(nu_i)
    st = lib().orc_run(C.byref(P), n, _ptr(pos), _ptr(vel), _ptr(ptype), int(nsteps),
                       _ptr(rs_), _ptr(nu_), _ptr(p), _ptr(fl), C.byref(it))
    if return_iters:
        return st, pos, vel, ptype, p, fl, int(it.value)
    return st, pos, vel, ptype, p, fl


def pressure_gradient(params, rs, ptype, p):
    """(status, phat[n], gradp[n][dim]) of a given pressure field at rs."""
    P, rs, ptype = _prep(params, rs, ptype)
    p = np.ascontiguousarray(p, dtype=np.float64)
    n, dim = rs.shape
    phat = np.zeros(n)
    gp = np.zeros((n, dim))
    L = lib()
    L.orc_pressure_gradient.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    st = L.orc_pressure_gradient(C.byref(P), n, _ptr(rs), _ptr(ptype), _ptr(p),
                                 _ptr(phat), _ptr(gp))
    return st, phat, gp


def pressure_update(params, rs, us, ptype, p, rho_s=None):
    """(status, pos[n][dim], vel[n][dim]): p-hat, gradient of a given pressure
    field at rs and the Euler update from the predicted state (rs, us)."""
    P, rs, ptype = _prep(params, rs, ptype)
    us = np.ascontiguousarray(us, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    n, dim = rs.shape
    pos = np.zeros((n, dim))
    vel = np.zeros((n, dim))
    L = lib()
    L.orc_pressure_update.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]
    st = L.orc_pressure_update(C.byref(P), n, _ptr(rs), _ptr(us), _ptr(ptype), _ptr(p),
                               _ptr(_opt(rho_s)), _ptr(pos), _ptr(vel))
    return st, pos, vel


def rollout_grad(params, pos, vel, ptype, nsteps, direction, w_ke=1.0, w_var=9.81, *,
                 rho_s=None, nu_i=None):
    """(status, L, dL/dnu, dL/dgx, <dL/du0, direction>) by dual numbers.
    Two-phase model: rho_s (smoothed densities) and nu_i; dL/dnu is then the
    derivative with respect to a common shift of all nu_i."""
    P, pos, ptype = _prep(params, pos, ptype)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    d = np.ascontiguousarray(direction, dtype=np.float64)
    rs_, nu_ = _opt(rho_s), _opt(nu_i)
    out = np.zeros(4)
    L = lib()
    L.orc_rollout_grad.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_double,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
    st = L.orc_rollout_grad(C.byref(P), pos.shape[0], _ptr(pos), _ptr(vel), _ptr(ptype),
                            int(nsteps), _ptr(d), float(w_ke), float(w_var), _ptr(rs_),
                            _ptr(nu_), _ptr(out))
    return st, out[0], out[1], out[2], out[3]


def loss(params, pos, vel, ptype, flags, w_ke=1.0, w_var=9.81):
    P, pos, ptype = _prep(params, pos, ptype)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    fl = np.ascontiguousarray(flags, dtype=np.int8)
    L = lib()
    L.orc_loss.argtypes = [C.POINTER(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_double, C.c_double]
    L.orc_loss.restype = C.c_double
    return L.orc_loss(C.byref(P), pos.shape[0], _ptr(pos), _ptr(vel), _ptr(ptype), _ptr(fl),
                      float(w_ke), float(w_var))


def smoothed_density(params, pos, ptype, rho_i):
    """(status, <rho>[n]) of the two-phase model."""
    P, pos, ptype = _prep(params, pos, ptype)
    r = np.ascontiguousarray(rho_i, dtype=np.float64)
    out = np.zeros(pos.shape[0])
    st = lib().orc_smoothed_density(C.byref(P), pos.shape[0], _ptr(pos), _ptr(ptype), _ptr(r),
                                    _ptr(out))
    return st, out
