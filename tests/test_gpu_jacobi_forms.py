"""The two forms of pca_jacobi_eigh (one workgroup holding the whole matrix,
and the block-cyclic form on many CUs) against the FP64 oracle, and a
workspace that holds stale or arbitrary bytes before a call."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import eig_err, report, sign_rule_holds

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EIG_TOL = 1e-5
ANGLE_TOL = 1e-4
# |V^T V - I|_max: the eigenvectors are products of float32 rotations, each
# orthogonal to about 2^-24, over sweeps * n rotations per column (a few
# 1e-5 at the larger band counts). A defect of e moves a vector by about e
# radians, so the eigenvector bound is also the bound that matters here.
ORTH_TOL = ANGLE_TOL


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


def eigh(P, A, form, tol=1e-6, max_sweeps=30, fp64_angles=True, ws=None, overlap=False):
    m = A.shape[0]
    Cd = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda()
    lam = torch.full((m,), float("nan"), dtype=torch.float32, device="cuda")
    V = torch.full((m, m), float("nan"), dtype=torch.float32, device="cuda")
    info = P.new_info()
    P.pca_jacobi_eigh(Cd, lam, V, tol, max_sweeps, fp64_angles, info, ws, overlap=overlap, form=form)
    return host(lam), host(V), P.read_info(info)


@pytest.mark.parametrize("form", ["block", "one_cu"])
@pytest.mark.parametrize("m", [2, 3, 16, 17, 31, 32, 33, 64, 100, 127, 128, 160, 224, 255, 256])
def test_forms_planted(pca, form, m):
    """Planted spectra over one block, several blocks, ragged last blocks and
    the largest band count."""
    say(f"jacobi {form} planted m={m}")
    rng = np.random.default_rng(300 + m)
    A, _, _ = synth.random_symmetric(rng, m, np.linspace(1.0, 0.05, m))
    A32 = A.astype(np.float32).astype(np.float64)
    ref_l, ref_V, _ = oracle.jacobi_eigh(A32)
    for fp64 in (True, False):
        lam, V, info = eigh(pca, A32, form, fp64_angles=fp64)
        say(f"  fp64_angles={fp64}: {info}")
        assert info["converged"] == 1 and info["nonfinite"] == 0, info
        assert eig_err(lam, ref_l) <= EIG_TOL
        r = report(lam, V, None, dict(lam=ref_l, V=ref_V, Q=None), m)
        assert r["angle"] <= ANGLE_TOL, r
        assert sign_rule_holds(V, list(range(m)))
        assert np.abs(V.astype(np.float64).T @ V - np.eye(m)).max() <= ORTH_TOL
        assert np.all(np.diff(lam) <= 0)


@pytest.mark.parametrize("form", ["block", "one_cu"])
def test_forms_special_inputs(pca, form):
    """Already diagonal (no rotation, zero sweeps), a zero row and column, a
    non-finite entry, a sweep limit, clustered and negative eigenvalues."""
    say(f"jacobi {form} special inputs")
    d = np.array([3.0, -1.0, 7.0, 0.5, 2.0] * 8)[:37] + np.arange(37) * 1e-3
    lam, V, info = eigh(pca, np.diag(d), form)
    assert info["sweeps"] == 0 and info["rotations"] == 0 and info["converged"] == 1, info
    assert np.array_equal(lam, np.sort(d.astype(np.float32))[::-1])
    assert np.array_equal(np.abs(V), np.eye(37)[:, np.argsort(-d.astype(np.float32), kind="stable")])
    rng = np.random.default_rng(3)
    A, _, _ = synth.random_symmetric(rng, 70)
    A[40, :] = 0.0
    A[:, 40] = 0.0
    ref_l, _, _ = oracle.jacobi_eigh(A.astype(np.float32).astype(np.float64))
    lam, V, info = eigh(pca, A, form)
    assert info["converged"] == 1 and eig_err(lam, ref_l) <= EIG_TOL
    B = np.eye(80)
    B[20, 63] = B[63, 20] = np.nan
    lam, V, info = eigh(pca, B, form)
    assert info["nonfinite"] == 1 and np.all(np.isnan(lam)), info
    A, _, _ = synth.random_symmetric(np.random.default_rng(4), 96)
    lam, V, info = eigh(pca, A, form, tol=1e-12, max_sweeps=1)
    assert info["sweeps"] == 1 and info["converged"] == 0, info
    # Clustered (pairs 1e-6 apart) and negative eigenvalues: eigenvalues only.
    spec = np.repeat(np.linspace(1.0, -0.5, 40), 2) + np.tile([0.0, 1e-6], 40)
    A, _, _ = synth.random_symmetric(np.random.default_rng(6), 80, spec)
    ref_l, _, _ = oracle.jacobi_eigh(A.astype(np.float32).astype(np.float64))
    lam, V, info = eigh(pca, A, form)
    assert info["converged"] == 1 and eig_err(lam, ref_l) <= EIG_TOL, info
    assert np.abs(V.astype(np.float64).T @ V - np.eye(80)).max() <= ORTH_TOL


def test_block_matches_one_cu_on_covariance(pca):
    """Both forms on the covariance of the 224-band cube: the same
    eigenvalues and leading eigenvectors within the tolerances."""
    d = synth.make_config("c3", n_pixels=1 << 15)
    Y = d["Y"].astype(np.float64)
    C = np.cov(Y, rowvar=False)
    ref_l, ref_V, _ = oracle.jacobi_eigh(C.astype(np.float32).astype(np.float64))
    for form in ("block", "one_cu"):
        lam, V, info = eigh(pca, C, form)
        r = report(lam, V, None, dict(lam=ref_l, V=ref_V, Q=None), 10)
        say(f"c3 covariance {form}: {info} {r}")
        assert info["converged"] == 1 and r["eig"] <= EIG_TOL and r["angle"] <= ANGLE_TOL, r


@pytest.mark.parametrize("form", ["block", "one_cu"])
def test_stale_workspace(pca, form):
    """A workspace that holds arbitrary bytes, then the log of a call on a
    different matrix: every call gives the same results as a call on a fresh
    zero-filled workspace (the overlapped replay included)."""
    m = 200
    A, _, _ = synth.random_symmetric(np.random.default_rng(11), m, np.linspace(2.0, 0.1, m))
    B, _, _ = synth.random_symmetric(np.random.default_rng(12), m, np.linspace(1.0, 0.3, m))
    nbytes = pca.pca_workspace_size(pca.PCA_OP_JACOBI, 2, m, max_sweeps=30)
    fresh = pca.workspace(nbytes)
    ref = eigh(pca, A, form, ws=fresh)
    ws = pca.workspace(nbytes)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    ws.copy_(torch.randint(0, 256, ws.shape, dtype=torch.uint8, device="cuda", generator=g))
    overlaps = (False, True) if form == "one_cu" else (False,)
    for ov in overlaps:
        got = eigh(pca, A, form, ws=ws, overlap=ov)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1]), ov
        eigh(pca, B, form, ws=ws, overlap=ov)                 # leaves B's log behind
        got = eigh(pca, A, form, ws=ws, overlap=ov)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1]), ov
        assert got[2]["steps"] == ref[2]["steps"]
