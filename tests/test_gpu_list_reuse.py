"""Neighbour lists kept over several steps (params skin > 0; Section
"Computational performance analysis": lists refreshed every few steps).
The cell search writes a superset at radius re_lap + skin, rebuilt when a
particle has moved skin/2 since the build; every step filters it to the
exact list (with one phase, inside the prediction kernel).  Bars: the exported list of every step is exactly the
definition's (all pairs, bit for bit); one step, including a step that
keeps its lists, against the oracle at the one-step bars; 20 FP64 steps at
the multi-step bar."""
import numpy as np
import pytest

from paper_2105_01677_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_01677_amd import mps
    return mps


def rel_err(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den else float(np.abs(a).max())


def _np(t):
    return t.detach().cpu().numpy()


def _cases(precision):
    w2 = W.with_skin(W.jitter(W.config("dam_break_2d_1432", precision=precision)), 0.5)
    w3 = W.with_skin(W.jitter(W.lattice_block(3, [14, 12, 10], walls_below=True, dt=2e-4,
                                              g=9.81)), 0.4)
    w3.params["precision"] = precision
    return [w2, w3]


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_kept_lists_are_the_fresh_lists(gpu, orc, precision):
    """After every step the lists a step would use (mps_neighbors) are
    exactly the all-pairs lists at the current positions, and the cells
    those of the current positions, while most steps keep their lists."""
    for w in _cases(precision):
        m = gpu.MPS(w.params, w.pos, w.vel, w.ptype)
        builds = 0
        nsteps = 30
        for k in range(nsteps):
            s = m.step(1)
            builds += s["list_builds"]
            cell, cnt, lst = (_np(x) for x in m.neighbors())
            st = {key: _np(v) for key, v in m.state().items()}
            so, cnt_o, lst_o = orc.neighbors_brute(w.params, st["pos"], st["type"])
            assert so == 0
            assert np.array_equal(cnt, cnt_o), (w.name, k)
            assert np.array_equal(lst, lst_o), (w.name, k)
            so, cell_o, _, _ = orc.neighbors_cells(w.params, st["pos"], st["type"])
            assert np.array_equal(cell, cell_o), (w.name, k)
        m.close()
        print(w.name, "list builds", builds, "of", nsteps, "steps", flush=True)
        assert 1 <= builds < nsteps // 2


@pytest.mark.parametrize("precond", [W.PC_JACOBI, W.PC_TWO_LEVEL, W.PC_BLOCK])
@pytest.mark.parametrize("precision,cg_tol,tol", [(W.FP64, 1e-12, 1e-8), (W.MIXED, 1e-9, 1e-4)])
def test_step_that_keeps_its_lists_against_the_oracle(gpu, orc, precision, cg_tol, tol, precond):
    """The second step (which keeps the first step's superset) against the
    oracle's step from the same state: displacement, velocity, pressure and
    number density at the one-step bars, flags equal outside the tie band.
    With the two-level preconditioner its aggregates are the cells of the
    last build, which the particle order follows; block Jacobi groups rows
    of that order (the solution is unique, so the bars are the same)."""
    for w in _cases(precision):
        w.params.update(cg_tol=cg_tol, precond=precond)
        m = gpu.MPS(w.params, w.pos, w.vel, w.ptype)
        m.step(1)
        s0 = {k: _np(v) for k, v in m.state().items()}
        s = m.step(1)
        assert s["list_builds"] == 0
        g = {k: _np(v) for k, v in m.state().items()}
        m.close()
        st, o = orc.step(w.params, s0["pos"], s0["vel"], s0["type"], want_lists=False)
        assert st == 0
        fw = (s0["type"] == W.FLUID) | (s0["type"] == W.WALL)
        if np.any((g["flags"] != o["flags"]) & fw):
            n0 = orc.lattice_constants(w.params["dim"], w.params["l0"], w.params["re_n"],
                                       w.params["kernel"])[0]
            mism = (g["flags"] != o["flags"]) & fw
            assert np.abs(o["nstar"][mism] / (w.params["beta"] * n0) - 1).max() < 2e-5
            st, o = orc.step(w.params, s0["pos"], s0["vel"], s0["type"],
                             flags_override=g["flags"], want_lists=False)
        errs = {"disp": rel_err(g["pos"] - s0["pos"], o["pos"] - s0["pos"]),
                "vel": rel_err(g["vel"], o["vel"]), "p": rel_err(g["p"], o["p"]),
                "nstar": rel_err(g["nstar"], o["nstar"])}
        print(w.name, errs, flush=True)
        for k, e in errs.items():
            assert e < tol, (w.name, k, e)


def test_twenty_steps_with_kept_lists_fp64(gpu, orc):
    w = W.with_skin(W.config("dam_break_2d_1432"), 0.5)
    w.params["cg_tol"] = 1e-12
    m = gpu.MPS(w.params, w.pos, w.vel, w.ptype)
    s = m.step(20)
    g = {k: _np(v) for k, v in m.state().items()}
    m.close()
    assert s["list_builds"] < 20
    st, pos, vel, t, p, fl = orc.run(w.params, w.pos, w.vel, w.ptype, 20)
    assert st == 0
    assert rel_err(g["pos"] - w.pos, pos - w.pos) < 1e-6
    assert rel_err(g["vel"], vel) < 1e-6
    assert rel_err(g["p"], p) < 1e-6


def test_skin_needs_cells_of_re_lap_plus_skin_and_no_adjoint(gpu):
    w = W.config("dam_break_2d_1432")
    bad = dict(w.params, skin=0.5 * w.params["l0"])
    with pytest.raises(gpu.MPSError):
        gpu.MPS(bad, w.pos, w.vel, w.ptype)
    ws = W.with_skin(w, 0.5)
    m = gpu.MPS(ws.params, ws.pos, ws.vel, ws.ptype)
    m.tape_alloc(2)
    m.tape_save(0)
    m.step(1)
    m.tape_load(0)
    import torch
    z = torch.zeros((w.n, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.MPSError):
        m.step_adjoint(z, z)
    m.close()


def test_dam_break_3d_kept_lists_stay_physical(gpu):
    """The 441,282-particle 3-D dam break over 100 steps with a skin of
    0.3 l0: no ghost, speeds physical, and fewer builds than steps."""
    w = W.with_skin(W.config("dam_break_3d_441282", precision=W.MIXED), 0.3)
    m = gpu.MPS(w.params, w.pos, w.vel, w.ptype)
    s = m.step(100)
    st = m.state()
    m.close()
    vel = _np(st["vel"])
    typ = _np(st["type"])
    vmax = float(np.linalg.norm(vel[typ == W.FLUID], axis=1).max())
    print("3-D kept lists: builds", s["list_builds"], "of 100, vmax", vmax, flush=True)
    assert (typ == W.GHOST).sum() == 0 and vmax < 5.0
    assert s["list_builds"] < 100


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_lists_filtered_by_the_prediction(gpu, orc, precision):
    """With kept lists and one phase the prediction kernel filters the
    superset into the step's exact lists (on the mixed path deciding on the
    FP32 records outside a band around the cut-off, on the FP64 positions
    inside it).  The entries of the lists a step used (the step's
    list_entries) equal the all-pairs count at the step's input positions,
    for a build step and for a step that keeps its lists; the plain lattice
    puts many pairs exactly at r = re_lap, inside the band."""
    w0 = W.with_skin(W.config("dam_break_2d_1432", precision=precision), 0.5)
    for w in [w0] + _cases(precision):
        m = gpu.MPS(w.params, w.pos, w.vel, w.ptype)
        s1 = m.step(1)
        st, cnt, _ = orc.neighbors_brute(w.params, w.pos, w.ptype)
        assert st == 0
        assert s1["list_entries"] == int(cnt.sum()), (w.name, s1["list_entries"], int(cnt.sum()))
        g = {k: _np(v) for k, v in m.state().items()}
        s2 = m.step(1)
        assert s2["list_builds"] == 0
        st, cnt, _ = orc.neighbors_brute(w.params, g["pos"], g["type"])
        assert st == 0
        assert s2["list_entries"] == int(cnt.sum()), (w.name, s2["list_entries"], int(cnt.sum()))
        m.close()
