"""Whole-step graphs of the PPE model: each step after the first is enqueued
as one graph with a CG iteration count guessed from the previous step, and
within one mps_step call the next step's graph is enqueued before the
previous step's result is read; a step whose solve needs more is discarded
(its input buffer is untouched) and redone with polled CG batches.  Every
way must give the same bits as the steps taken with direct, polled launches
(profiling mode runs no graphs)."""
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


def _run(mps, w, steps, graphs, maxit=None, per_call=1):
    prm = dict(w.params)
    if maxit is not None:
        prm["cg_maxit"] = maxit
    m = mps.MPS(prm, w.pos, w.vel, w.ptype)
    if not graphs:
        m.profile(["cg_spmv"])
    stats = [m.step(per_call, allow_noconv=True) for _ in range(steps // per_call)]
    st = m.state()
    out = {k: st[k].detach().cpu().numpy() for k in ("pos", "vel", "p", "flags")}
    m.close()
    return out, stats


@pytest.mark.parametrize("precond", [W.PC_JACOBI, W.PC_BLOCK])
@pytest.mark.parametrize("precision", [W.MIXED, W.FP64])
def test_speculative_steps_match_polled(gpu, precision, precond):
    w = W.jitter(W.config("dam_break_2d_1432", precision=precision))
    w.params["precond"] = precond
    a, sa = _run(gpu, w, 30, True)
    b, sb = _run(gpu, w, 30, False)
    assert [s["cg_iters_last"] for s in sa] == [s["cg_iters_last"] for s in sb]
    assert all(s["status"] == gpu.OK for s in sa)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precond", [W.PC_JACOBI, W.PC_BLOCK])
@pytest.mark.parametrize("precision", [W.MIXED, W.FP64])
def test_pipelined_steps_match_polled(gpu, precision, precond):
    """30 steps in one call (two step graphs in flight) against 30 polled
    single steps, and against 3 calls of 10."""
    w = W.jitter(W.config("dam_break_2d_1432", precision=precision))
    w.params["precond"] = precond
    a, sa = _run(gpu, w, 30, True, per_call=30)
    b, _ = _run(gpu, w, 30, False)
    c, _ = _run(gpu, w, 30, True, per_call=10)
    assert sa[0]["status"] == gpu.OK and sa[0]["steps"] == 30
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(c[k], b[k]), k


@pytest.mark.parametrize("precond", [W.PC_JACOBI, W.PC_BLOCK])
def test_speculative_step_redone_when_solve_needs_more(gpu, precond):
    # the solve is capped below what it needs: every speculative step after
    # the first fails to converge, is discarded and redone, and ends with
    # the capped iterate like the polled path
    w = W.jitter(W.config("dam_break_2d_1432"))
    w.params["precond"] = precond
    a, sa = _run(gpu, w, 5, True, maxit=12)
    b, sb = _run(gpu, w, 5, False, maxit=12)
    assert all(s["status"] == gpu.E_CG_NOCONV for s in sa + sb)
    assert [s["cg_redone"] for s in sa] == [0, 1, 1, 1, 1]
    assert all(s["cg_redone"] == 0 for s in sb)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # the same five steps in one call: steps 2-5 fail inside the pipeline
    p, sp = _run(gpu, w, 5, True, maxit=12, per_call=5)
    assert sp[0]["status"] == gpu.E_CG_NOCONV and sp[0]["cg_redone"] == 4
    for k in a:
        assert np.array_equal(p[k], b[k]), k


def test_dam_break_3d_runs_physical(gpu):
    """The 441,282-particle 3-D dam break over its first 100 steps (one call:
    pipelined step graphs, split CG with predicated slot loads): every solve
    converges, no particle leaves the grid, and the fluid stays below
    10 sqrt(2 g H); the falling column has picked up speed."""
    w = W.config("dam_break_3d_441282")
    m = gpu.MPS(w.params, w.pos, w.vel, w.ptype)
    s = m.step(100)
    st = m.state()
    vel = st["vel"].cpu().numpy()
    typ = st["type"].cpu().numpy()
    m.close()
    assert s["status"] == gpu.OK and s["steps"] == 100 and s["n_ghost"] == 0
    assert 20 < s["cg_iters_total"] / 100 < 80
    f0 = w.ptype == W.FLUID
    h = float(w.pos[f0, 2].max() - w.pos[f0, 2].min())
    speed = np.linalg.norm(vel[typ == W.FLUID], axis=1)
    assert np.isfinite(vel).all()
    assert speed.max() < 10 * np.sqrt(2 * 9.81 * h)
    assert speed.max() > 0.1       # g t = 0.196 m/s after 100 steps of 2e-4 s


def _ring_scene(pmode, precision):
    """A ring of fluid particles converging on a particle at its centre, in
    the air of the 2-D tank: the centre's list outgrows the cap at a known
    step (the eighth in the oracle as well), every earlier step clean.  For
    the PPE model the resting water column stays beside it (its solve keeps
    the whole-step graphs in use; the ring's pressure stays mild); for the
    equation of state the ring is alone, 24 particles against a cap of 20,
    so that its spacing stays above l0 and its pressure at zero."""
    w = W.config("dam_break_2d_1432", pmode=pmode, precision=precision)
    dt, l0 = w.params["dt"], w.params["l0"]
    c = np.array([0.5, 0.45])
    m, speed, cap = (64, 0.5, 50) if pmode == W.PPE_CG else (24, 0.45, 20)
    ang = 2 * np.pi * np.arange(m) / m
    e = np.stack([np.cos(ang), np.sin(ang)], 1)
    ring, rv = c + 7 * l0 * e, -speed * l0 / dt * e
    if pmode == W.PPE_CG:
        pos = np.vstack([w.pos, ring, c[None]])
        vel = np.vstack([w.vel, rv, [[0.0, 0.0]]])
        typ = np.concatenate([w.ptype, np.zeros(m + 1, np.int8)])
    else:
        pos, vel = np.vstack([ring, c[None]]), np.vstack([rv, [[0.0, 0.0]]])
        typ = np.zeros(m + 1, np.int8)
    return dict(w.params, max_neigh=cap), pos, vel, typ


def _state(m):
    st = m.state()
    return {k: st[k].detach().cpu().numpy() for k in ("pos", "vel", "p", "type")}


@pytest.mark.parametrize("precision", [W.MIXED, W.FP64])
@pytest.mark.parametrize("pmode", [W.PPE_CG, W.WC_EOS])
def test_error_stops_at_the_failing_step(gpu, pmode, precision):
    """An error raised in step k of a call ends the call there: the status
    names it, stats.steps counts the k - 1 steps completed before it, and
    the context's state is step k's input, bit for bit as after k - 1 clean
    steps.  PPE: whole-step graphs, two in flight; EOS: graphs of two steps
    with no host synchronisation in between."""
    prm, pos, vel, typ = _ring_scene(pmode, precision)
    m = gpu.MPS(prm, pos, vel, typ)
    before = []
    for k in range(1, 12):
        st, _ = m.step_status(1)
        if st != gpu.OK:
            break
        before.append(_state(m))
    m.close()
    assert st == gpu.E_NEIGH_OVERFLOW
    k_fail = len(before) + 1
    assert k_fail == 8
    for done in (0, 3):
        m = gpu.MPS(prm, pos, vel, typ)
        if done:
            assert m.step_status(done)[0] == gpu.OK
        st, stats = m.step_status(10)
        assert st == gpu.E_NEIGH_OVERFLOW
        assert stats["steps"] == k_fail - 1 - done
        got = _state(m)
        for key, a in before[k_fail - 2].items():
            assert np.array_equal(got[key], a), (done, key)
        # poisoned until the state is set again
        assert m.step_status(1)[0] == gpu.E_POISONED
        m.close()
