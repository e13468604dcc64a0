"""Whole-step graphs of the PPE model: each step after the first is enqueued
as one graph with a CG iteration count guessed from the previous step; a
step whose solve needs more is discarded (its input buffer is untouched)
and redone with polled CG batches.  Both must give the same bits as the
steps taken with direct, polled launches (profiling mode runs no graphs)."""
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


def _run(mps, w, steps, graphs, maxit=None):
    prm = dict(w.params)
    if maxit is not None:
        prm["cg_maxit"] = maxit
    m = mps.MPS(prm, w.pos, w.vel, w.ptype)
    if not graphs:
        m.profile(["cg_spmv"])
    stats = [m.step(1, allow_noconv=True) for _ in range(steps)]
    st = m.state()
    out = {k: st[k].detach().cpu().numpy() for k in ("pos", "vel", "p", "flags")}
    m.close()
    return out, stats


@pytest.mark.parametrize("precision", [W.MIXED, W.FP64])
def test_speculative_steps_match_polled(gpu, precision):
    w = W.jitter(W.config("cfg1", precision=precision))
    a, sa = _run(gpu, w, 30, True)
    b, sb = _run(gpu, w, 30, False)
    assert [s["cg_iters_last"] for s in sa] == [s["cg_iters_last"] for s in sb]
    assert all(s["status"] == gpu.OK for s in sa)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_speculative_step_redone_when_solve_needs_more(gpu):
    # the solve is capped below what it needs: every speculative step after
    # the first fails to converge, is discarded and redone, and ends with
    # the capped iterate like the polled path
    w = W.jitter(W.config("cfg1"))
    a, sa = _run(gpu, w, 5, True, maxit=12)
    b, sb = _run(gpu, w, 5, False, maxit=12)
    assert all(s["status"] == gpu.E_CG_NOCONV for s in sa + sb)
    assert [s["cg_redone"] for s in sa] == [0, 1, 1, 1, 1]
    assert all(s["cg_redone"] == 0 for s in sb)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
