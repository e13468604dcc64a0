"""The block-Jacobi preconditioner's definiteness (host side, on the
oracle's matrices).  The library applies one damped Neumann step of block
Jacobi over groups of 64 consecutive cell-sorted rows,
M^-1 = D^-1/2 (I - omega N) D^-1/2 with N = D^-1/2 (A_B - D) D^-1/2 and
omega = 1.5; it is symmetric positive definite while omega lambda_max(N) < 1.
These tests build A from the oracle (rows ordered by cell, as the GPU path
orders them), and check the bound with a margin on the workloads the
preconditioner serves (2-D and 3-D, the kernel and the Eq. 23 Laplacians),
plus the plain facts the argument rests on: N has a zero diagonal and
non-positive entries, and every row of D^-1 (A_B - D) sums to at most 1 in
absolute value (weak diagonal dominance)."""
import numpy as np
import pytest

from paper_2105_01677_amd import workloads as W

OMEGA = 1.5    # the library's damping factor of the block-Jacobi step
GROUP = 64     # rows per group (one fused workgroup)


def _grouped_system(orc, w):
    st, o = orc.step(dict(w.params, clamp=0), w.pos, w.vel, w.ptype, want_matrix=True)
    assert st == 0
    n = w.n
    order = np.lexsort((np.arange(n), o["cell"]))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    inner = np.nonzero(o["flags"] == 0)[0]
    inner = inner[np.argsort(rank[inner])]
    idx = -np.ones(n, np.int64)
    idx[inner] = np.arange(len(inner))
    m = len(inner)
    d = o["diag"][inner]
    AB = np.zeros((m, m))     # off-diagonal entries inside a row's group
    full = np.zeros(m)        # sum |a_ij| over all off-diagonal entries
    for r, i in enumerate(inner):
        c = o["count"][i]
        for j, a in zip(o["list"][i, :c], o["aval"][i, :c]):
            if a == 0.0 or idx[j] < 0:
                continue
            full[r] += abs(a)
            if rank[i] // GROUP == rank[j] // GROUP:
                AB[r, idx[j]] += a
    return d, AB, full


@pytest.mark.parametrize("laplacian,bound", [(W.LAP_STD, 0.3), (W.LAP_HL, 0.5)])
def test_block_jacobi_is_definite_2d(orc, laplacian, bound):
    w = W.jitter(W.config("dam_break_2d_1432"))
    w.params.update(laplacian=laplacian)
    d, AB, full = _grouped_system(orc, w)
    assert np.all(d > 0)
    assert np.all(np.diag(AB) == 0) and np.all(AB <= 0)
    assert np.allclose(AB, AB.T, rtol=1e-12, atol=0)
    assert np.all(full <= d * (1 + 1e-12))
    s = 1 / np.sqrt(d)
    N = s[:, None] * AB * s[None, :]
    lam = np.linalg.eigvalsh(N)
    print("2-D laplacian", laplacian, "lambda range", lam[0], lam[-1], flush=True)
    assert lam[-1] < bound and OMEGA * lam[-1] < 0.75
    # the preconditioner itself: symmetric with positive eigenvalues
    Minv = (np.diag(1 / d) - OMEGA * (AB / d[:, None]) / d[None, :])
    assert np.allclose(Minv, Minv.T, rtol=1e-12, atol=0)
    assert np.linalg.eigvalsh(Minv).min() > 0


@pytest.mark.parametrize("laplacian", [W.LAP_STD, W.LAP_HL])
def test_block_jacobi_is_definite_3d(orc, laplacian):
    w = W.jitter(W.lattice_block(3, [12, 10, 10], walls_below=True, dt=2e-4))
    w.params.update(laplacian=laplacian)
    d, AB, full = _grouped_system(orc, w)
    assert np.all(AB <= 0) and np.all(full <= d * (1 + 1e-12))
    s = 1 / np.sqrt(d)
    lam = np.linalg.eigvalsh(s[:, None] * AB * s[None, :])
    print("3-D laplacian", laplacian, "lambda range", lam[0], lam[-1], flush=True)
    assert OMEGA * lam[-1] < 0.5


def test_damping_past_the_bound_loses_definiteness(orc):
    """The check has teeth: far enough past 1 / lambda_max the same
    construction is indefinite."""
    w = W.jitter(W.config("dam_break_2d_1432"))
    d, AB, _ = _grouped_system(orc, w)
    s = 1 / np.sqrt(d)
    lmax = np.linalg.eigvalsh(s[:, None] * AB * s[None, :])[-1]
    om = 1.2 / lmax
    Minv = (np.diag(1 / d) - om * (AB / d[:, None]) / d[None, :])
    assert np.linalg.eigvalsh(Minv).min() < 0
