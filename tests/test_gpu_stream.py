"""PCAStream: several cubes in flight on separate HIP streams give, for every
cube, exactly the result of the one-cube pipeline (same kernels, same
chunking, so bitwise), and match the FP64 oracle."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import report, SUBSPACE_TOL

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
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("chain", [False, True])
def test_stream_matches_single_pipeline(pca, chain):
    n, m, k = 20000, 96, 6
    cubes = [synth.mixture_cube(np.random.default_rng(900 + i), n, m, 6, 1.0, 0.01) for i in range(3)]
    Yd = [torch.from_numpy(c).cuda() for c in cubes]
    ref = []
    for Y in Yd:
        r = pca.PCAPipeline(n, m, k, "bf16x3", jacobi="one_cu").forward(Y)   # the stream's eigen-solver form
        ref.append([host(t).copy() for t in (r.mean, r.eigvals, r.V, r.Q)])
    ps = pca.PCAStream(n, m, k, "bf16x3", depth=2, chain=chain)
    # Seven submissions over two slots: every slot is reused while the other
    # is still in flight; check each result once its event has completed.
    for i in range(7):
        r, ev = ps.submit(Yd[i % 3])
        ev.synchronize()
        got = [host(t) for t in (r.mean, r.eigvals, r.V, r.Q)]
        assert all(np.array_equal(a, b) for a, b in zip(got, ref[i % 3])), i
        assert pca.read_info(r.info)["converged"] == 1
    ps.join()
    torch.cuda.synchronize()
    for i, Y in enumerate(cubes):
        rep = report(ref[i][1], ref[i][2], ref[i][3], oracle.pca(Y, k), k)
        say(f"stream cube {i}: eig {rep['eig']:.2e} angle {rep['angle']:.2e}")
        assert rep["eig"] <= 1e-5 and rep["angle"] <= 1e-4
        assert rep.get("subspace", 0.0) <= SUBSPACE_TOL, rep


def test_stream_overlapped_results(pca):
    """Results read only after all cubes are queued (slots overlap in time)."""
    n, m, k = 30000, 128, 8
    cubes = [synth.mixture_cube(np.random.default_rng(950 + i), n, m, 8, 0.5, 0.005) for i in range(4)]
    Yd = [torch.from_numpy(c).cuda() for c in cubes]
    ps = pca.PCAStream(n, m, k, "f32", depth=4)
    res = [ps.submit(Y)[0] for Y in Yd]
    ps.join()
    torch.cuda.synchronize()
    for i, (Y, r) in enumerate(zip(Yd, res)):
        s = pca.PCAPipeline(n, m, k, "f32", jacobi="one_cu").forward(Y)
        assert np.array_equal(host(s.eigvals), host(r.eigvals)), i
        assert np.array_equal(host(s.Q), host(r.Q)), i


def test_stream_rejects_bad_shape(pca):
    ps = pca.PCAStream(100, 8, 2, depth=2)
    with pytest.raises(ValueError):
        ps.submit(torch.zeros(100, 9, device="cuda"))
    with pytest.raises(ValueError):
        pca.PCAStream(100, 8, 2, depth=0)
