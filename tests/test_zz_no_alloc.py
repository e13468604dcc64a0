"""The allocation-free neighbour search (mps_neighbors_noalloc) against the
context's mps_neighbors on the same positions: cell ids, counts and lists
bit for bit, over calls in a row whose later inputs are smaller (the fixed
scratch array keeps the earlier call's data), plus its error paths."""
import numpy as np
import pytest

from paper_2105_01677_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2105_01677_amd import mps
    mps.lib()
    return torch


def _context_lists(w):
    from paper_2105_01677_amd import mps
    m = mps.MPS(w.params, w.pos, w.vel, w.ptype)
    cell, cnt, lst = m.neighbors()
    out = (cell.cpu().numpy(), cnt.cpu().numpy(), lst.cpu().numpy())
    m.close()
    return out


def _noalloc_lists(w):
    from paper_2105_01677_amd import mps
    cell, cnt, lst = mps.neighbors_noalloc(w.params, w.pos, w.ptype)
    return cell.cpu().numpy(), cnt.cpu().numpy(), lst.cpu().numpy()


def test_noalloc_matches_mps_neighbors_over_calls_in_a_row(gpu, orc):
    from paper_2105_01677_amd import mps
    cases = [W.jitter(W.config("dam_break_2d_44832")),
             W.jitter(W.config("dam_break_2d_1432")),
             W.random_box(3000, 3)]
    for k, w in enumerate(cases):
        print(f"noalloc call {k}: {w.name} n={w.n}", flush=True)
        ref = _context_lists(w)
        gpu.cuda.synchronize()
        free0 = gpu.cuda.mem_get_info()[0]
        got = _noalloc_lists(w)
        if k > 0:
            # the call itself allocates nothing on the device (the outputs
            # are torch's, allocated before the free memory is read)
            pos = gpu.as_tensor(w.pos, dtype=gpu.float64).cuda()
            typ = gpu.as_tensor(w.ptype, dtype=gpu.int8).cuda()
            outs = (gpu.empty(w.n, dtype=gpu.int32, device="cuda"),
                    gpu.empty(w.n, dtype=gpu.int32, device="cuda"),
                    gpu.empty((w.n, w.params["max_neigh"]), dtype=gpu.int32, device="cuda"))
            gpu.cuda.synchronize()
            free1 = gpu.cuda.mem_get_info()[0]
            mps.neighbors_noalloc(w.params, pos, typ, out=outs)
            gpu.cuda.synchronize()
            assert gpu.cuda.mem_get_info()[0] == free1
            for a, b in zip(outs, got):
                assert np.array_equal(a.cpu().numpy(), b)
        for name, a, b in zip(("cell", "count", "list"), got, ref):
            assert np.array_equal(a, b), (w.name, name)
        del free0
    # the small 2-D case also against the definition (all pairs)
    w = cases[1]
    st, cnt_o, lst_o = orc.neighbors_brute(w.params, w.pos, w.ptype)
    assert st == 0
    got = _noalloc_lists(w)
    assert np.array_equal(got[1], cnt_o) and np.array_equal(got[2], lst_o)


def test_noalloc_error_paths(gpu):
    from paper_2105_01677_amd import mps
    # more than the fixed array holds: refused before any launch
    w = W.random_box(200_000, 2)
    need = 200_000 * (16 * 2 + 30 + 4 * 304)
    assert need > mps.NOALLOC_SCRATCH_BYTES
    with pytest.raises(mps.MPSError) as e:
        mps.neighbors_noalloc(w.params, w.pos, w.ptype)
    assert e.value.status == mps.E_SCRATCH and "scratch" in str(e.value)
    # too small a cap: the kernels' own bound raises the overflow status
    w = W.jitter(W.config("dam_break_2d_1432"))
    prm = dict(w.params, max_neigh=8)
    with pytest.raises(mps.MPSError) as e:
        mps.neighbors_noalloc(prm, w.pos, w.ptype)
    assert e.value.status == mps.E_NEIGH_OVERFLOW
    # an invalid particle type
    t = w.ptype.copy()
    t[5] = 7
    with pytest.raises(mps.MPSError) as e:
        mps.neighbors_noalloc(w.params, w.pos, t)
    assert e.value.status == mps.E_ARG
    # and a valid call after the errors is exact again
    ref = _context_lists(w)
    got = _noalloc_lists(w)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
