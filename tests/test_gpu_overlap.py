"""pca_jacobi_eigh with PCA_JACOBI_OVERLAP_REPLAY (the eigenvectors formed by
workgroups that follow the rotation log while the sweeps run) against the
same call without it: the same arithmetic in the same order, so the results
must agree bit for bit; plus the oracle on the end-to-end path that uses it."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import eig_err, report, SUBSPACE_TOL

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


class Eigh:
    """Buffers and one workspace for repeated pca_jacobi_eigh calls."""

    def __init__(self, P, m, max_sweeps=30):
        self.P, self.m, self.max_sweeps = P, m, max_sweeps
        self.lam = torch.empty(m, dtype=torch.float32, device="cuda")
        self.V = torch.empty(m, m, dtype=torch.float32, device="cuda")
        self.info = P.new_info()
        self.ws = P.workspace(P.pca_workspace_size(P.PCA_OP_JACOBI, 2, m, max_sweeps=max_sweeps))

    def __call__(self, Cd, overlap, tol=1e-6, fp64_angles=True):
        self.lam.fill_(float("nan"))
        self.V.fill_(float("nan"))
        self.P.pca_jacobi_eigh(Cd, self.lam, self.V, tol, self.max_sweeps, fp64_angles, self.info, self.ws,
                               overlap=overlap)
        return host(self.lam), host(self.V), self.P.read_info(self.info)


def same(a, b):
    return np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("m", [2, 3, 7, 33, 64, 127, 224, 256])
def test_overlap_bitwise(pca, m):
    """Odd and even band counts, one and several follower workgroups, the
    largest band count; three overlapped calls in a row on one workspace
    (the progress record's epoch advances) interleaved with plain calls."""
    rng = np.random.default_rng(900 + m)
    A, _, _ = synth.random_symmetric(rng, m, np.linspace(1.0, 0.02, m))
    Cd = torch.from_numpy(A.astype(np.float32)).cuda()
    e = Eigh(pca, m)
    lam0, V0, info0 = e(Cd, overlap=False)
    for rep in range(3):
        lam1, V1, info1 = e(Cd, overlap=True)
        say(f"m={m} rep {rep}: sweeps {info1['sweeps']} steps {info1['steps']}")
        assert same(lam0, lam1) and same(V0, V1), rep
        assert info1 == info0
        lam2, V2, _ = e(Cd, overlap=False)
        assert same(lam0, lam2) and same(V0, V2)
    ref_l, _, _ = oracle.jacobi_eigh(A.astype(np.float32).astype(np.float64))
    assert eig_err(lam1, ref_l) <= 1e-5
    assert np.abs(V1.astype(np.float64).T @ V1 - np.eye(m)).max() <= 1e-5


def test_overlap_degenerate_runs(pca):
    """No step at all (a diagonal matrix; max_sweeps = 0), one sweep only,
    float32 angles, and a non-finite input (the Jacobi workgroup publishes
    an empty log and the NaN result is reported as before)."""
    e = Eigh(pca, 6)
    d = np.diag([3.0, -1.0, 7.0, 0.5, 2.0, 1.0]).astype(np.float32)
    Cd = torch.from_numpy(d).cuda()
    for ov in (False, True):
        lam, V, info = e(Cd, overlap=ov)
        assert info["steps"] == 0 and np.array_equal(lam, np.sort(np.diag(d))[::-1])
    A, _, _ = synth.random_symmetric(np.random.default_rng(5), 40)
    Ad = torch.from_numpy(A.astype(np.float32)).cuda()
    e0 = Eigh(pca, 40, max_sweeps=0)
    r0, r1 = e0(Ad, False), e0(Ad, True)
    assert r1[2]["steps"] == 0 and same(r0[0], r1[0]) and same(r0[1], r1[1])
    e1 = Eigh(pca, 40, max_sweeps=1)
    r0, r1 = e1(Ad, False, tol=1e-12), e1(Ad, True, tol=1e-12)
    assert r1[2]["sweeps"] == 1 and same(r0[0], r1[0]) and same(r0[1], r1[1])
    r0, r1 = e1(Ad, False, fp64_angles=False), e1(Ad, True, fp64_angles=False)
    assert same(r0[0], r1[0]) and same(r0[1], r1[1])
    B = np.eye(6, dtype=np.float32)
    B[2, 3] = B[3, 2] = np.nan
    lam, V, info = e(torch.from_numpy(B).cuda(), overlap=True)
    assert info["nonfinite"] == 1 and np.all(np.isnan(lam))
    # The workspace is ready for the next call after a non-finite input.
    lam, V, info = e(Cd, overlap=True)
    assert info["nonfinite"] == 0 and np.array_equal(lam, np.sort(np.diag(d))[::-1])


def test_overlap_pipeline_oracle_and_graph(pca):
    """The whole pipeline with the overlapped replay (the PCAPipeline
    default) against the oracle, against the plain replay bitwise, and
    captured in a HIP graph replayed several times with eager work between
    the replays."""
    d = synth.make_config("c2")
    k = d["k"]
    Yh = d["Y"]
    Yd = torch.from_numpy(Yh).cuda()
    n, m = Yh.shape
    ov = pca.PCAPipeline(n, m, k, "bf16x3")
    assert ov.overlap_replay
    plain = pca.PCAPipeline(n, m, k, "bf16x3", overlap_replay=False)
    r_ov, r_pl = ov.forward(Yd), plain.forward(Yd)
    outs = [host(t) for t in (r_ov.eigvals, r_ov.V, r_ov.Q)]
    assert all(same(a, host(b)) for a, b in zip(outs, (r_pl.eigvals, r_pl.V, r_pl.Q)))
    ref = oracle.pca(Yh, k)
    r = report(outs[0], outs[1], outs[2], ref, k)
    say(f"c2 overlapped: {r}")
    assert r["eig"] <= 1e-5 and r["angle"] <= 1e-4 and r["proj"] <= 1e-4
    assert r.get("subspace", 0.0) <= SUBSPACE_TOL, r
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ov.forward(Yd)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        ov.forward(Yd)
    for rep in range(3):
        for t in (ov.eigvals, ov.V, ov.Q):
            t.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        got = [host(t) for t in (ov.eigvals, ov.V, ov.Q)]
        assert all(same(a, b) for a, b in zip(outs, got)), rep
        ov.forward(Yd)   # an eager call between replays advances the same record
        torch.cuda.synchronize()
        assert all(same(a, host(b)) for a, b in zip(outs, (ov.eigvals, ov.V, ov.Q))), rep
