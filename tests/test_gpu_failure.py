"""Bounded waits that run out, forced from the host (pca_set_wait_shift
shortens every wait bound of the Jacobi kernels): each kernel still ends,
the call reports a non-finite result (the block-cyclic form's step barrier)
or NaN eigenvector rows (the followers of the overlapped replay and of the
batched form), and the next call with the default bounds is bitwise the
same as before."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pca():
    import paper_2403_18321_amd as P
    P.library()
    return P


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().copy()


def eigh(P, A, form, overlap=False):
    m = A.shape[0]
    Cd = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    lam = torch.full((m,), float("nan"), dtype=torch.float32, device="cuda")
    V = torch.full((m, m), float("nan"), dtype=torch.float32, device="cuda")
    info = P.new_info()
    P.pca_jacobi_eigh(Cd, lam, V, 1e-6, 30, True, info, overlap=overlap, form=form)
    return host(lam), host(V), P.read_info(info)


def shortened(P, fn):
    """fn() with every wait bound divided by 2^40 (restored afterwards)."""
    P.set_wait_shift(40)
    try:
        return fn()
    finally:
        P.set_wait_shift(0)


def test_block_barrier_runs_out(pca):
    A, _, _ = synth.random_symmetric(np.random.default_rng(21), 200, np.linspace(2.0, 0.1, 200))
    ref = eigh(pca, A, "block")
    assert ref[2]["converged"] == 1
    lam, V, info = shortened(pca, lambda: eigh(pca, A, "block"))
    say(f"block form, shortened waits: {info}")
    assert info["nonfinite"] == 1 and info["converged"] == 0, info
    assert np.all(np.isnan(lam)) and np.all(np.isnan(V))
    again = eigh(pca, A, "block")
    assert np.array_equal(again[0], ref[0]) and np.array_equal(again[1], ref[1])


def test_overlap_followers_run_out(pca):
    A, _, _ = synth.random_symmetric(np.random.default_rng(22), 200, np.linspace(2.0, 0.1, 200))
    ref = eigh(pca, A, "one_cu", overlap=True)
    lam, V, info = shortened(pca, lambda: eigh(pca, A, "one_cu", overlap=True))
    rows = int(np.isnan(V).any(axis=1).sum())
    say(f"one-CU form, overlapped replay, shortened waits: {info}, NaN rows {rows}")
    assert rows > 0
    again = eigh(pca, A, "one_cu", overlap=True)
    assert np.array_equal(again[0], ref[0]) and np.array_equal(again[1], ref[1])


def test_batched_followers_run_out(pca):
    cubes = [synth.mixture_cube(np.random.default_rng(800 + i), n, m, 4, 1.0, 0.01)
             for i, (n, m) in enumerate([(3000, 120), (2000, 64), (4000, 200)])]
    Yd = [torch.from_numpy(Y).cuda() for Y in cubes]
    b = pca.BatchedPCA(Yd, 3, "f32")
    b.run()
    ref = [host(v) for v in b.V]

    def run():
        for v in b.V:
            v.fill_(0.0)
        b.run()
        return [host(v) for v in b.V]

    got = shortened(pca, run)
    nan_rows = sum(int(np.isnan(v).any(axis=1).sum()) for v in got)
    say(f"batched form, shortened waits: NaN eigenvector rows {nan_rows}")
    assert nan_rows > 0
    again = run()
    assert all(np.array_equal(a, r) for a, r in zip(again, ref))
