"""Seeded synthetic inputs for the MPS hot path: particle geometry, types,
initial velocities and physical parameters.

This module holds no arithmetic of the method itself (no kernel weights, no
n0/lambda, no neighbour search): it only lays particles on lattices, assigns
their types and fills a parameter dictionary.  Both the HIP path and the test
oracle consume what it produces, so it is the single source of inputs.

Geometry follows the usual MPS dam-break set-up of the paper (Section
"Dam break"): fluid particles on a square/cubic lattice of spacing l0 with
centres at (i + 1/2) l0 from the tank's inner corner, and boundary layers k =
1..L at distance (k - 1/2) l0 outside each wall.  The first layers are wall
particles (pressure unknowns, Listing "PPE assemble GPU code" treats them like
fluid), the outer layers dummy particles (only in number-density and viscous
sums; excluded from the PPE).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FLUID, WALL, DUMMY, GHOST = 0, 1, 2, 3
PPE_CG, WC_EOS = 0, 1
K_KOSHIZUKA, K_CUBIC = 0, 1
FP64, MIXED = 0, 1
GRAD_STD, GRAD_CMPS = 0, 1
SRC_STD, SRC_HS, SRC_HS_ECS = 0, 1, 2
LAP_STD, LAP_HL = 0, 1
PC_JACOBI, PC_TWO_LEVEL, PC_BLOCK = 0, 1, 2

SEED = 2105


def default_params(dim: int, l0: float, *, re_n_over_l0: float = 2.1,
                   re_lap_over_l0: float | None = None, pmode: int = PPE_CG,
                   kernel: int | None = None, dt: float = 5e-4,
                   rho: float = 1000.0, nu: float = 1e-6, g: float = 9.81,
                   c0: float = 20.0, precision: int = FP64) -> dict:
    """Physical and numerical parameters as a plain dict.

    Defaults: beta = 0.97 (free-surface criterion, Eq. 15), gamma = 7 (Eq. 16),
    alpha = 1e-7 artificial compressibility on the PPE diagonal (Listing "PPE
    assemble GPU code"), neighbour cap 300 (Section "CUDA").  The kernel
    defaults to Eq. 4 for the PPE and to the cubic kernel for the equation of
    state, as the paper recommends for each pressure model.
    """
    if re_lap_over_l0 is None:
        re_lap_over_l0 = 4.0 if dim == 2 else 3.1
    if kernel is None:
        kernel = K_KOSHIZUKA if pmode == PPE_CG else K_CUBIC
    gvec = [0.0, -g, 0.0] if dim == 2 else [0.0, 0.0, -g]
    return dict(
        dim=dim, l0=l0, re_n=re_n_over_l0 * l0, re_lap=re_lap_over_l0 * l0,
        rho=rho, nu=nu, g=gvec, dt=dt, beta=0.97, c0=c0, gamma=7.0,
        alpha=1e-7, cg_tol=1e-9, cg_maxit=10000, max_neigh=300,
        pmode=pmode, kernel=kernel, precision=precision, grad=GRAD_STD,
        clamp=1, smag_cs=0.0, cg_pipelined=1, source=SRC_STD, laplacian=LAP_STD, skin=0.0,
        precond=PC_JACOBI,
        grid_lo=[0.0, 0.0, 0.0], grid_n=[1, 1, 1], cell_size=0.0,
    )


@dataclasses.dataclass
class Workload:
    name: str
    pos: np.ndarray      # [n, dim] float64
    vel: np.ndarray      # [n, dim] float64
    ptype: np.ndarray    # [n] int8
    params: dict
    steps: int = 1
    rho_i: np.ndarray | None = None   # [n] per-particle density (two-phase)
    nu_i: np.ndarray | None = None    # [n] per-particle viscosity (two-phase)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def counts(self) -> dict:
        t = self.ptype
        return {"fluid": int((t == FLUID).sum()), "wall": int((t == WALL).sum()),
                "dummy": int((t == DUMMY).sum()), "total": self.n}


def _tank_particles(dim, l0, inner, fill, n_wall, n_dummy, closed_top):
    """Lattice particles for a rectangular tank.

    inner: inner tank size per axis (m); fill: fluid block size per axis (m),
    anchored at the inner corner.  Returns (pos, type) with fluid first, then
    boundary particles in lattice order.
    """
    ni = [int(round(inner[a] / l0)) for a in range(dim)]
    nf = [int(round(fill[a] / l0)) for a in range(dim)]
    nl = n_wall + n_dummy
    # fluid
    axes = [np.arange(nf[a]) for a in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    fidx = np.stack([gr.ravel() for gr in grids], axis=1)
    # boundary: all lattice sites of the padded box not inside the tank
    up = dim - 1
    lo_i = [-nl] * dim
    hi_i = [ni[a] + nl for a in range(dim)]
    if not closed_top:
        hi_i[up] = ni[up]          # open top: walls up to the tank-top height
    axes = [np.arange(lo_i[a], hi_i[a]) for a in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    bidx = np.stack([gr.ravel() for gr in grids], axis=1)
    outside = np.zeros(len(bidx), dtype=np.int64)
    for a in range(dim):
        below = np.maximum(-bidx[:, a], 0)
        above = np.maximum(bidx[:, a] - (ni[a] - 1), 0)
        if a == up and not closed_top:
            above = np.zeros_like(above)
        outside = np.maximum(outside, np.maximum(below, above))
    keep = outside > 0
    bidx, layer = bidx[keep], outside[keep]
    btype = np.where(layer <= n_wall, WALL, DUMMY).astype(np.int8)
    pos = np.concatenate([fidx, bidx]).astype(np.float64)
    pos = (pos + 0.5) * l0
    ptype = np.concatenate([np.full(len(fidx), FLUID, np.int8), btype])
    return pos, ptype, ni, nl


def _set_grid(params, pos, l0, ni, nl, headroom_cells):
    """Fixed background grid: cell side slightly above re_lap so that a pair
    closer than re_lap can never land two cells apart through rounding of
    the cell-coordinate arithmetic; one padding cell around the particles and
    extra head-room cells above an open top."""
    dim = params["dim"]
    cs = params["re_lap"] * (1.0 + 2.0 ** -20)
    lo, n = [0.0, 0.0, 0.0], [1, 1, 1]
    for a in range(dim):
        lo_a = -nl * l0 - cs
        hi_a = (ni[a] + nl) * l0 + cs
        if a == dim - 1:
            hi_a += headroom_cells * cs
        lo[a] = lo_a
        n[a] = int(math.ceil((hi_a - lo_a) / cs))
    params["grid_lo"], params["grid_n"], params["cell_size"] = lo, n, cs


def with_skin(w: Workload, skin_over_l0: float) -> Workload:
    """The same workload with neighbour lists kept over steps: a skin of
    skin_over_l0 * l0 and grid cells enlarged to re_lap + skin (same lower
    corner, at least the same extent)."""
    prm = dict(w.params)
    skin = skin_over_l0 * prm["l0"]
    cs = (prm["re_lap"] + skin) * (1.0 + 2.0 ** -20)
    ext = [prm["grid_n"][a] * prm["cell_size"] for a in range(3)]
    prm["grid_n"] = [max(1, int(math.ceil(ext[a] / cs))) if a < prm["dim"] else 1
                     for a in range(3)]
    prm["cell_size"] = cs
    prm["skin"] = skin
    return dataclasses.replace(w, params=prm)


def wc_dt(l0: float, c0: float, dt: float) -> float:
    """Time step of the explicit weakly-compressible model: the requested dt,
    capped at an acoustic Courant number c0 dt / l0 of 0.8 (at 1.6 the 2-D
    dam break at l0 = 1.25 mm blows up within 100 steps)."""
    return min(dt, 0.8 * l0 / c0)


def dam_break_2d(l0=0.01, *, tank=(0.8, 0.6), column=(0.2, 0.3), pmode=PPE_CG,
                 dt=None, steps=200, precision=FP64, c0=20.0) -> Workload:
    """2-D dam break: water column 0.2 x 0.3 m in a 0.8 x 0.6 m open tank,
    2 wall + 2 dummy layers (Section "Dam break" set-up)."""
    if dt is None:
        dt = 5e-4 if l0 >= 0.01 else 1e-4
    if pmode == WC_EOS:
        dt = wc_dt(l0, c0, dt)
    pos, ptype, ni, nl = _tank_particles(2, l0, tank, column, 2, 2, False)
    prm = default_params(2, l0, pmode=pmode, dt=dt, precision=precision, c0=c0)
    _set_grid(prm, pos, l0, ni, nl, headroom_cells=2)
    vel = np.zeros_like(pos)
    return Workload(f"dam_break_2d_l0={l0}", pos, vel, ptype, prm, steps)


def dam_break_3d(l0=0.007, *, tank=(1.6, 0.6, 0.6), block=(0.4, 0.6, 0.3),
                 pmode=PPE_CG, dt=2e-4, steps=500, precision=MIXED) -> Workload:
    """3-D dam break: 0.4 x 0.6 x 0.3 m block in a 1.6 x 0.6 x 0.6 m open
    tank, 1 wall + 2 dummy layers."""
    pos, ptype, ni, nl = _tank_particles(3, l0, tank, block, 1, 2, False)
    prm = default_params(3, l0, pmode=pmode, dt=dt, precision=precision)
    _set_grid(prm, pos, l0, ni, nl, headroom_cells=2)
    vel = np.zeros_like(pos)
    return Workload(f"dam_break_3d_l0={l0}", pos, vel, ptype, prm, steps)


def sloshing_2d(l0=0.002, *, tank=(0.6, 0.3), depth=0.15, amp=0.05,
                dt=1e-4, steps=500, precision=MIXED, jitter=0.01) -> Workload:
    """2-D sloshing tank with the first standing-wave mode as initial
    velocity (divergence-free, zero normal velocity at the walls):
    u = A sin(kx) cosh(ky)/cosh(kh), v = -A cos(kx) sinh(ky)/cosh(kh),
    k = pi/L.  A seeded 1 % amplitude jitter makes the field generic."""
    pos, ptype, ni, nl = _tank_particles(2, l0, tank, (tank[0], depth), 2, 2, False)
    prm = default_params(2, l0, pmode=WC_EOS, dt=wc_dt(l0, 20.0, dt), precision=precision)
    _set_grid(prm, pos, l0, ni, nl, headroom_cells=2)
    k = math.pi / tank[0]
    rng = np.random.default_rng(SEED)
    vel = np.zeros_like(pos)
    f = ptype == FLUID
    x, y = pos[f, 0], pos[f, 1]
    a = amp * (1.0 + jitter * rng.uniform(-1, 1, size=x.shape))
    vel[f, 0] = a * np.sin(k * x) * np.cosh(k * y) / math.cosh(k * depth)
    vel[f, 1] = -a * np.cos(k * x) * np.sinh(k * y) / math.cosh(k * depth)
    return Workload(f"sloshing_2d_l0={l0}", pos, vel, ptype, prm, steps)


def two_phase_3d(l0=0.005, *, box=(0.5, 0.5, 1.0), amp=0.01, steps=200,
                 dt=2e-4, precision=MIXED) -> Workload:
    """3-D closed box, heavy liquid (rho 1500, nu 1e-5) over light liquid
    (rho 1000, nu 1e-6) with a perturbed interface
    z = H/2 + amp cos(2 pi x / Lx) cos(2 pi y / Ly); 1 wall + 2 dummy layers
    on all six faces; Smagorinsky constant 0.12."""
    pos, ptype, ni, nl = _tank_particles(3, l0, box, box, 1, 2, True)
    prm = default_params(3, l0, pmode=PPE_CG, dt=dt, precision=precision,
                         rho=1000.0, nu=1e-6)
    prm["smag_cs"] = 0.12
    _set_grid(prm, pos, l0, ni, nl, headroom_cells=0)
    rng = np.random.default_rng(SEED)
    vel = np.zeros_like(pos)
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    a = amp * (1.0 + 0.01 * rng.uniform(-1, 1))
    zi = 0.5 * box[2] + a * np.cos(2 * math.pi * x / box[0]) * np.cos(2 * math.pi * y / box[1])
    heavy = z >= zi
    rho_i = np.where(heavy, 1500.0, 1000.0)
    nu_i = np.where(heavy, 1e-5, 1e-6)
    return Workload(f"two_phase_3d_l0={l0}", pos, vel, ptype, prm, steps,
                    rho_i=rho_i, nu_i=nu_i)


def water_drop(l0=0.05, *, radius=1.0, strain=100.0, c0=1000.0, dt=1e-5,
               precision=FP64, steps=1000) -> Workload:
    """2-D elliptic water drop (Section "Water drop"): fluid particles on the
    square lattice points (i l0, j l0) with i^2 + j^2 <= (R/l0)^2, no walls,
    no gravity, initial velocity (-A x, A y) with A = 100 1/s; the weakly-
    compressible model with the cubic kernel and re = 3 l0 for every sum,
    dt = 1e-5 s, rho = 1000, nu = 1e-6.  The printed radius and spacing do
    not give the printed 1,257 particles; R = 1 m at l0 = 0.05 m gives
    exactly that count (lattice points of the closed disc).  c0 is not
    printed: 1,000 m/s (Mach 0.1 at the initial 100 m/s, acoustic Courant
    number 0.2).  The grid spans the square of side 5 R around the drop,
    which holds the ellipse up to b = 2.5 R."""
    m = int(math.floor(radius / l0 + 1e-9))
    ii = np.arange(-m, m + 1)
    I, J = np.meshgrid(ii, ii, indexing="ij")
    keep = I * I + J * J <= m * m
    pos = np.stack([I[keep], J[keep]], axis=1).astype(np.float64) * l0
    vel = np.stack([-strain * pos[:, 0], strain * pos[:, 1]], axis=1)
    ptype = np.full(len(pos), FLUID, np.int8)
    prm = default_params(2, l0, re_n_over_l0=3.0, re_lap_over_l0=3.0, pmode=WC_EOS,
                         kernel=K_CUBIC, dt=dt, g=0.0, c0=c0, precision=precision)
    cs = prm["re_lap"] * (1.0 + 2.0 ** -20)
    half = 2.5 * radius + cs
    n = int(math.ceil(2.0 * half / cs))
    prm["grid_lo"], prm["grid_n"], prm["cell_size"] = [-half, -half, 0.0], [n, n, 1], cs
    return Workload("water_drop_2d", pos, vel, ptype, prm, steps)


def drop_axes(pos: np.ndarray) -> tuple[float, float]:
    """Semi-axes (a along x, b along y) of an elliptic drop from the second
    moments of its particle positions about their mean: a uniform ellipse
    has <x^2> = a^2/4 and <y^2> = b^2/4."""
    c = pos - pos.mean(axis=0)
    return 2.0 * math.sqrt(float((c[:, 0] ** 2).mean())), 2.0 * math.sqrt(float((c[:, 1] ** 2).mean()))


def jitter(w: Workload, *, pos_amp=0.05, vel_sigma=0.05, seed=SEED) -> Workload:
    """Parity inputs: fluid positions jittered uniformly by +-pos_amp*l0 and
    fluid velocities drawn from N(0, vel_sigma) m/s, so that every term of
    the step (viscous, density deviation, pressure) is exercised."""
    rng = np.random.default_rng(seed)
    l0 = w.params["l0"]
    pos, vel = w.pos.copy(), w.vel.copy()
    f = w.ptype == FLUID
    pos[f] += rng.uniform(-pos_amp * l0, pos_amp * l0, size=pos[f].shape)
    vel[f] += rng.normal(0.0, vel_sigma, size=vel[f].shape)
    return dataclasses.replace(w, name=w.name + "+jitter", pos=pos, vel=vel,
                               params=dict(w.params))


def random_box(n, dim, *, l0=0.01, seed=SEED, re_lap_over_l0=None) -> Workload:
    """Uniformly random particles (all fluid) in a cube sized for roughly
    lattice density; used for neighbour-search parity on unstructured input."""
    rng = np.random.default_rng(seed)
    side = (n ** (1.0 / dim)) * l0
    pos = rng.uniform(0.0, side, size=(n, dim))
    prm = default_params(dim, l0, re_lap_over_l0=re_lap_over_l0)
    ni = [int(math.ceil(side / l0))] * dim
    _set_grid(prm, pos, l0, ni, 0, headroom_cells=0)
    vel = np.zeros_like(pos)
    ptype = np.zeros(n, np.int8)
    return Workload(f"random_box_{dim}d_n={n}", pos, vel, ptype, prm, 1)


def config(name: str, **kw) -> Workload:
    """The five benchmark workloads, named by case and particle count: the
    2-D dam break at 1,432 and 44,832, the 3-D dam break at 441,282, the
    2-D sloshing tank at 24,932 and the 3-D two-phase box at 2,314,616."""
    if name == "dam_break_2d_1432":
        return dam_break_2d(0.01, dt=kw.pop("dt", 5e-4), steps=200, **kw)
    if name == "dam_break_2d_44832":
        # The plain method (Eq. 13 source, Eq. 7 Laplacian) blows up on this
        # case near step 274 at dt = 1e-4 (the FP64 oracle as well as the
        # GPU); with the HS source and the HL Laplacian (source=SRC_HS,
        # laplacian=LAP_HL) it runs all 1,000 steps.
        return dam_break_2d(0.00125, dt=kw.pop("dt", 1e-4), steps=1000, **kw)
    if name == "dam_break_3d_441282":
        return dam_break_3d(0.007, **kw)
    if name == "sloshing_2d_24932":
        return sloshing_2d(0.002, **kw)
    if name == "two_phase_3d_2314616":
        return two_phase_3d(0.005, **kw)
    raise KeyError(name)


def lattice_block(dim: int, m, *, l0=0.01, pmode=PPE_CG, dt=5e-4, g=0.0,
                  walls_below: bool = False) -> Workload:
    """A free block of m[0] x m[1] (x m[2]) fluid particles on the lattice,
    optionally resting on 2 wall + 2 dummy layers; zero velocity.  Deep
    interior particles see a perfect lattice, which the closed-form pins of
    the oracle rely on."""
    m = [m] * dim if isinstance(m, int) else list(m)
    axes = [np.arange(m[a]) for a in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    idx = np.stack([gr.ravel() for gr in grids], axis=1)
    ptype = np.full(len(idx), FLUID, np.int8)
    nl = 0
    if walls_below:
        nl = 4
        axes = [np.arange(-nl, m[a] + nl) for a in range(dim - 1)] + [np.arange(-nl, 0)]
        grids = np.meshgrid(*axes, indexing="ij")
        bidx = np.stack([gr.ravel() for gr in grids], axis=1)
        layer = -bidx[:, dim - 1]
        idx = np.concatenate([idx, bidx])
        ptype = np.concatenate([ptype, np.where(layer <= 2, WALL, DUMMY).astype(np.int8)])
    pos = (idx.astype(np.float64) + 0.5) * l0
    prm = default_params(dim, l0, pmode=pmode, dt=dt, g=g)
    _set_grid(prm, pos, l0, m, nl, headroom_cells=2)
    return Workload(f"lattice_block_{dim}d", pos, np.zeros_like(pos), ptype, prm, 1)
