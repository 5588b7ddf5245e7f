"""pca_jacobi_eigh_noalloc (the library's own device array as the
workspace) against pca_jacobi_eigh with a workspace argument: the same
kernels on the same input, so the results agree bit for bit; two calls in a
row, the second on a smaller matrix, for both Jacobi forms."""

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


def run(P, A, noalloc, form, overlap=False, max_sweeps=30):
    m = A.shape[0]
    Cd = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    lam = torch.full((m,), float("nan"), dtype=torch.float32, device="cuda")
    V = torch.full((m, m), float("nan"), dtype=torch.float32, device="cuda")
    info = P.new_info()
    if noalloc:
        P.pca_jacobi_eigh_noalloc(Cd, lam, V, 1e-6, max_sweeps, True, info, overlap=overlap, form=form)
    else:
        ws = P.workspace(P.pca_workspace_size(P.PCA_OP_JACOBI, 2, m, max_sweeps=max_sweeps))
        P.pca_jacobi_eigh(Cd, lam, V, 1e-6, max_sweeps, True, info, ws, overlap=overlap, form=form)
    return host(lam), host(V), P.read_info(info)


@pytest.mark.parametrize("form,overlap", [("block", False), ("one_cu", False), ("one_cu", True)])
def test_noalloc_matches_workspace_call(pca, form, overlap):
    for m, seed in ((224, 41), (64, 42)):
        say(f"noalloc {form} overlap={overlap} m={m}")
        A, _, _ = synth.random_symmetric(np.random.default_rng(seed), m, np.linspace(1.0, 0.05, m))
        ref = run(pca, A, False, form, overlap)
        got = run(pca, A, True, form, overlap)
        assert ref[2]["converged"] == 1 and got[2] == ref[2], (got[2], ref[2])
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])


def test_noalloc_refuses_oversized_request(pca):
    A = np.eye(256, dtype=np.float32)
    with pytest.raises(pca.PCAError):
        run(pca, A, True, "block", max_sweeps=100000)
