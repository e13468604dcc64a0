"""Python binding of the HIP MPS library (include/mps.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libmps_hip.so.  PyTorch provides device memory and the stream.  There is
no fallback: if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmps_hip.so")

OK, E_ARG, E_NOMEM, E_NEIGH_OVERFLOW, E_CG_NOCONV = 0, -1, -2, -3, -4
E_NONFINITE, E_COINCIDENT, E_DEVICE, E_POISONED, E_SCRATCH = -5, -6, -7, -8, -9
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_NOMEM", -3: "E_NEIGH_OVERFLOW",
                -4: "E_CG_NOCONV", -5: "E_NONFINITE", -6: "E_COINCIDENT",
                -7: "E_DEVICE", -8: "E_POISONED", -9: "E_SCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 << 20


class MPSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("pmode", C.c_int32), ("kernel", C.c_int32),
        ("precision", C.c_int32), ("grad", C.c_int32), ("clamp_negative_p", C.c_int32),
        ("max_neigh", C.c_int32), ("cg_maxit", C.c_int32), ("grid_n", C.c_int32 * 3),
        ("cg_pipelined", C.c_int32),
        ("l0", C.c_double), ("re_n", C.c_double), ("re_lap", C.c_double),
        ("rho", C.c_double), ("nu", C.c_double), ("g", C.c_double * 3),
        ("dt", C.c_double), ("beta", C.c_double), ("c0", C.c_double),
        ("gamma", C.c_double), ("alpha", C.c_double), ("cg_tol", C.c_double),
        ("grid_lo", C.c_double * 3), ("cell_size", C.c_double),
        ("smagorinsky_cs", C.c_double), ("source", C.c_int32), ("laplacian", C.c_int32),
        ("skin", C.c_double), ("precond", C.c_int32),
    ]


class StepStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("cg_iters_last", C.c_int32),
                ("cg_iters_total", C.c_int64), ("cg_relres_last", C.c_double),
                ("n_surface", C.c_int64), ("n_ghost", C.c_int64),
                ("list_entries", C.c_int64), ("ppe_nnz", C.c_int64),
                ("cg_redone", C.c_int32), ("list_builds", C.c_int32),
                ("short_entries", C.c_int64)]


_lib = None
_VP = C.c_void_p


def lib() -> C.CDLL:
    """Load libmps_hip.so (built by paper_2105_01677_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run build())")
        L = C.CDLL(LIB_PATH)
        L.mps_init.argtypes = [C.POINTER(Params), C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP,
                               C.POINTER(_VP)]
        L.mps_free.argtypes = [_VP]
        L.mps_last_error.argtypes = [_VP]
        L.mps_last_error.restype = C.c_char_p
        L.mps_neighbors.argtypes = [_VP, _VP, _VP, _VP]
        L.mps_neighbors_noalloc.argtypes = [C.POINTER(Params), C.c_int64, _VP, _VP, _VP, _VP,
                                            _VP, _VP]
        L.mps_step.argtypes = [_VP, C.c_int32, C.POINTER(StepStats)]
        L.mps_pressure_solve.argtypes = [_VP, _VP, _VP, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double)]
        L.mps_get_ppe.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP]
        L.mps_get_state.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP]
        L.mps_set_state.argtypes = [_VP, _VP, _VP, _VP]
        L.mps_get_phase.argtypes = [_VP, _VP, _VP]
        L.mps_device_bytes.argtypes = [_VP, C.POINTER(C.c_int64)]
        L.mps_tape_alloc.argtypes = [_VP, C.c_int32]
        L.mps_tape_save.argtypes = [_VP, C.c_int32]
        L.mps_tape_load.argtypes = [_VP, C.c_int32]
        L.mps_step_adjoint.argtypes = [_VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_double), _VP]
        L.mps_profile.argtypes = [_VP, C.c_uint32]
        L.mps_profile_read.argtypes = [_VP, _VP, _VP]
        L.mps_constants.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        for f in ("mps_init", "mps_free", "mps_neighbors", "mps_step", "mps_pressure_solve",
                  "mps_get_ppe", "mps_get_state", "mps_set_state", "mps_constants",
                  "mps_profile", "mps_profile_read", "mps_tape_alloc", "mps_tape_save",
                  "mps_tape_load", "mps_step_adjoint", "mps_get_phase", "mps_device_bytes",
                  "mps_neighbors_noalloc"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


EXPORTED = ["mps_init", "mps_free", "mps_last_error", "mps_neighbors", "mps_step",
            "mps_pressure_solve", "mps_get_ppe", "mps_get_state", "mps_set_state",
            "mps_constants", "mps_profile", "mps_profile_read", "mps_tape_alloc",
            "mps_tape_save", "mps_tape_load", "mps_step_adjoint", "mps_get_phase",
            "mps_device_bytes", "mps_neighbors_noalloc"]

KERNEL_CLASSES = ["sort", "neighbors", "predict", "density", "assemble", "cg_spmv",
                  "cg_update", "gradient"]


def make_params(p: dict) -> Params:
    o = Params()
    o.dim, o.pmode, o.kernel = int(p["dim"]), int(p["pmode"]), int(p["kernel"])
    o.precision, o.grad = int(p["precision"]), int(p["grad"])
    o.clamp_negative_p = int(p["clamp"])
    o.max_neigh, o.cg_maxit = int(p["max_neigh"]), int(p["cg_maxit"])
    o.cg_pipelined = int(p.get("cg_pipelined", 0))
    for k in ("l0", "re_n", "re_lap", "rho", "nu", "dt", "beta", "c0", "gamma", "alpha",
              "cg_tol", "cell_size"):
        setattr(o, k, float(p[k]))
    o.smagorinsky_cs = float(p.get("smag_cs", 0.0))
    o.source = int(p.get("source", 0))
    o.laplacian = int(p.get("laplacian", 0))
    o.skin = float(p.get("skin", 0.0))
    o.precond = int(p.get("precond", 0))
    for a in range(3):
        o.g[a] = float(p["g"][a])
        o.grid_lo[a] = float(p["grid_lo"][a])
        o.grid_n[a] = int(p["grid_n"][a])
    return o


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(x, dtype):
    """A contiguous device tensor of the given dtype from numpy or torch."""
    import torch
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.detach().to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to("cuda")


def neighbors_noalloc(params: dict, pos, ptype, *, out=None, stream=None):
    """mps_neighbors_noalloc: cell ids, counts and lists (original ids,
    ascending, padded with -1) of the particles at pos, without a context;
    the library allocates nothing (its work arrays live in a fixed device
    array).  out: optional (cell [n] int32, count [n] int32, list
    [n][max_neigh] int32) device tensors to write, else allocated here by
    torch.  stream: a torch stream (default: the current one)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the MPS library needs a HIP device")
    pos = _dev(pos, torch.float64)
    typ = _dev(ptype, torch.int8)
    n = pos.shape[0]
    K = int(params["max_neigh"])
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device="cuda"),
               torch.empty(n, dtype=torch.int32, device="cuda"),
               torch.empty((n, K), dtype=torch.int32, device="cuda"))
    cell, cnt, lst = out
    P = make_params(params)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().mps_neighbors_noalloc(C.byref(P), n, _ptr(pos), _ptr(typ), _ptr(cell),
                                     _ptr(cnt), _ptr(lst), C.c_void_p(s.cuda_stream))
    if st != OK:
        raise MPSError(st, "mps_neighbors_noalloc: " + lib().mps_last_error(None).decode())
    return cell, cnt, lst


class MPS:
    """One simulation context on the current CUDA (HIP) device and stream."""

    def __init__(self, params: dict, pos, vel, ptype, rho_i=None, nu_i=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the MPS library needs a HIP device")
        self.torch = torch
        self.params = dict(params)
        self.pos0 = _dev(pos, torch.float64)
        vel0 = _dev(vel, torch.float64)
        t0 = _dev(ptype, torch.int8)
        if self.pos0.ndim != 2 or vel0.shape != self.pos0.shape or t0.shape != (self.pos0.shape[0],):
            raise MPSError(E_ARG, "pos/vel must be [n][dim] and type [n]")
        self.n, self.dim = self.pos0.shape
        if self.dim != params["dim"]:
            raise MPSError(E_ARG, f"pos has {self.dim} columns but dim = {params['dim']}")
        # a dedicated stream (default priority): the library captures its step
        # stages into HIP graphs, which the legacy default stream cannot hold
        self.stream = torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        self._P = make_params(params)
        h = C.c_void_p()
        r_i = _dev(rho_i, torch.float64)
        n_i = _dev(nu_i, torch.float64)
        self.stream.wait_stream(torch.cuda.current_stream())
        st = lib().mps_init(C.byref(self._P), self.n, _ptr(self.pos0), _ptr(vel0), _ptr(t0),
                            _ptr(r_i), _ptr(n_i), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise MPSError(st, "mps_init failed")
        self.h = h
        self.K = int(params["max_neigh"])

    def _check(self, st, what):
        if st != OK:
            msg = lib().mps_last_error(self.h).decode()
            raise MPSError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            lib().mps_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def constants(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self._check(lib().mps_constants(self.h, C.byref(a), C.byref(b), C.byref(c)),
                    "mps_constants")
        return a.value, b.value, c.value

    def step_status(self, nsteps: int = 1):
        """mps_step without raising: (status, statistics).  After an error,
        statistics["steps"] is the number of steps completed before the
        failing one, and the state is that step's input."""
        s = StepStats()
        st = lib().mps_step(self.h, int(nsteps), C.byref(s))
        return st, {"status": st, "steps": s.steps, "cg_iters_last": s.cg_iters_last,
                    "cg_iters_total": s.cg_iters_total, "cg_relres_last": s.cg_relres_last,
                    "n_surface": s.n_surface, "n_ghost": s.n_ghost,
                    "list_entries": s.list_entries, "ppe_nnz": s.ppe_nnz,
                    "cg_redone": s.cg_redone, "list_builds": s.list_builds,
                    "short_entries": s.short_entries}

    def step(self, nsteps: int = 1, *, allow_noconv=False) -> dict:
        st, stats = self.step_status(nsteps)
        if not (allow_noconv and st == E_CG_NOCONV):
            self._check(st, "mps_step")
        return stats

    def profile(self, classes):
        """Time every launch of the named kernel classes with HIP events."""
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
        self._check(lib().mps_profile(self.h, mask), "mps_profile")

    def profile_read(self) -> dict:
        ms = (C.c_double * len(KERNEL_CLASSES))()
        n = (C.c_int64 * len(KERNEL_CLASSES))()
        self._check(lib().mps_profile_read(self.h, ms, n), "mps_profile_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def device_bytes(self) -> int:
        b = C.c_int64()
        self._check(lib().mps_device_bytes(self.h, C.byref(b)), "mps_device_bytes")
        return b.value

    def phase(self):
        """(smoothed density, eddy viscosity) of a two-phase context."""
        torch = self.torch
        r = torch.empty(self.n, dtype=torch.float64, device="cuda")
        nt = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self._check(lib().mps_get_phase(self.h, _ptr(r), _ptr(nt)), "mps_get_phase")
        return r, nt

    def tape_alloc(self, nslots: int):
        self._check(lib().mps_tape_alloc(self.h, int(nslots)), "mps_tape_alloc")

    def tape_save(self, slot: int):
        self._check(lib().mps_tape_save(self.h, int(slot)), "mps_tape_save")

    def tape_load(self, slot: int):
        self._check(lib().mps_tape_load(self.h, int(slot)), "mps_tape_load")

    def step_adjoint(self, pos_bar, vel_bar):
        """Cotangents of the current step's input from those of its output:
        returns (pos_bar_prev, vel_bar_prev, nu_bar, g_bar[dim])."""
        torch = self.torch
        pb = _dev(pos_bar, torch.float64)
        vb = _dev(vel_bar, torch.float64)
        pp = torch.empty_like(pb)
        vp = torch.empty_like(vb)
        nub = C.c_double()
        gb = (C.c_double * 3)()
        self.stream.wait_stream(torch.cuda.current_stream())
        self._check(lib().mps_step_adjoint(self.h, _ptr(pb), _ptr(vb), _ptr(pp), _ptr(vp),
                                           C.byref(nub), gb), "mps_step_adjoint")
        return pp, vp, nub.value, [gb[a] for a in range(self.dim)]

    def step_raw(self, nsteps: int) -> int:
        """mps_step without statistics; returns the status."""
        return lib().mps_step(self.h, int(nsteps), None)

    def neighbors(self):
        torch = self.torch
        cell = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cnt = torch.empty(self.n, dtype=torch.int32, device="cuda")
        lst = torch.empty((self.n, self.K), dtype=torch.int32, device="cuda")
        self._check(lib().mps_neighbors(self.h, _ptr(cell), _ptr(cnt), _ptr(lst)),
                    "mps_neighbors")
        return cell, cnt, lst

    def pressure_solve(self, rhs=None):
        torch = self.torch
        p = torch.empty(self.n, dtype=torch.float64, device="cuda")
        rhs = _dev(rhs, torch.float64)
        self.stream.wait_stream(torch.cuda.current_stream())
        it, rr = C.c_int32(), C.c_double()
        st = lib().mps_pressure_solve(self.h, _ptr(rhs), _ptr(p), C.byref(it), C.byref(rr))
        self._check(st, "mps_pressure_solve")
        return p, it.value, rr.value

    def get_ppe(self):
        torch = self.torch
        d = torch.empty(self.n, dtype=torch.float64, device="cuda")
        b = torch.empty(self.n, dtype=torch.float64, device="cuda")
        nnz = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cols = torch.empty((self.n, self.K), dtype=torch.int32, device="cuda")
        vals = torch.empty((self.n, self.K), dtype=torch.float64, device="cuda")
        self._check(lib().mps_get_ppe(self.h, _ptr(d), _ptr(b), _ptr(nnz), _ptr(cols),
                                      _ptr(vals)), "mps_get_ppe")
        return {"diag": d, "b": b, "nnz": nnz, "cols": cols, "vals": vals}

    def state(self) -> dict:
        torch = self.torch
        out = {
            "pos": torch.empty((self.n, self.dim), dtype=torch.float64, device="cuda"),
            "vel": torch.empty((self.n, self.dim), dtype=torch.float64, device="cuda"),
            "p": torch.empty(self.n, dtype=torch.float64, device="cuda"),
            "nstar": torch.empty(self.n, dtype=torch.float64, device="cuda"),
            "flags": torch.empty(self.n, dtype=torch.int8, device="cuda"),
            "type": torch.empty(self.n, dtype=torch.int8, device="cuda"),
        }
        self._check(lib().mps_get_state(self.h, *[_ptr(out[k]) for k in
                                                  ("pos", "vel", "p", "nstar", "flags", "type")]),
                    "mps_get_state")
        return out

    def set_state(self, pos, vel, ptype=None):
        torch = self.torch
        pos = _dev(pos, torch.float64)
        vel = _dev(vel, torch.float64)
        t = _dev(ptype, torch.int8)
        self.stream.wait_stream(torch.cuda.current_stream())
        self._check(lib().mps_set_state(self.h, _ptr(pos), _ptr(vel), _ptr(t)), "mps_set_state")
