"""GPU path (through the C ABI) against the FP64 oracle on the same bytes."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import eig_err, report, sign_rule_holds, SUBSPACE_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EIG_TOL = 1e-5      # normwise eigenvalue error
ANGLE_TOL = 1e-4    # radians, well-separated eigenvectors
PROJ_TOL = 1e-4     # relative, per well-separated projection column
# Covariance entries, relative to max |C|: float32 and the exact 16-bit split
# (bf16x4) keep float32 rounding (~1e-7 per entry after the float64 chunk
# combination); bf16x3 also drops lo*lo, a bias of up to ~2^-16 of a diagonal
# entry. The float16 split (fp16x3) holds about 22 bits of each scaled value
# and drops lo*lo (together under 3 * 2^-22 of |x_i x_j| per product), on top
# of the float32 accumulation of the other forms.
COV_TOL = {"f32": 2e-6, "bf16x4": 2e-6, "bf16x3": 3e-5, "fp16x3": 3e-6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pca():
    import paper_2403_18321_amd as P
    P.library()
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_cov(P, Y, mode="f32", centered=False):
    n, m = Y.shape
    C = torch.empty(m, m, dtype=torch.float32, device="cuda")
    mean = torch.empty(m, dtype=torch.float32, device="cuda")
    P.pca_covariance(Y, C, None if centered else mean, P.COV_MODES[mode], centered)
    return host(C), (None if centered else host(mean))


@pytest.mark.parametrize("m", [2, 3, 5, 31, 32, 33, 64, 100, 127, 128, 200, 224, 255, 256])
def test_covariance_shapes(pca, m):
    say(f"covariance shape test m={m}")
    rng = np.random.default_rng(100 + m)
    n = 1000 + 13 * m
    Yh = synth.mixture_cube(rng, n, m, 4, 1.0, 0.01)
    ref = oracle.pca(Yh, 1)
    Yd = dev(Yh)
    for mode in ("f32", "bf16x3", "bf16x4", "fp16x3"):
        C, mean = gpu_cov(pca, Yd, mode)
        scale = np.abs(ref["C"]).max()
        err = np.abs(C - ref["C"]).max() / scale
        assert err <= COV_TOL[mode], (mode, err)
        assert np.array_equal(C, C.T), "covariance not exactly symmetric"
        assert np.abs(mean - ref["mean"]).max() <= 1e-6 * np.abs(ref["mean"]).max()


def test_covariance_strided_and_u16(pca):
    say("covariance strided / uint16")
    rng = np.random.default_rng(7)
    n, m = 5000, 60
    u = synth.radiance_cube_u16(rng, n, m, 5, 1.0)
    ref = oracle.pca(u, 1)
    for mode in ("f32", "bf16x3", "bf16x4", "fp16x3"):
        C, mean = gpu_cov(pca, dev(u), mode)
        assert np.abs(C - ref["C"]).max() / np.abs(ref["C"]).max() <= COV_TOL[mode], mode
        assert np.abs(mean - ref["mean"]).max() <= 1e-6 * ref["mean"].max()
    # Row stride larger than the band count (a view of a wider array).
    wide = np.zeros((n, m + 7), dtype=np.float32)
    wide[:, :m] = u.astype(np.float32)
    Yd = dev(wide)[:, :m]
    C, mean = gpu_cov(pca, Yd, "f32")
    assert np.abs(C - ref["C"]).max() / np.abs(ref["C"]).max() <= COV_TOL["f32"]


@pytest.mark.parametrize("n,m,pad", [(1000, 8, 0), (3001, 96, 0), (20001, 224, 0), (4099, 256, 8), (2500, 104, 16)])
def test_covariance_u16_rows_staged_in_lds(pca, n, m, pad):
    """uint16 cubes whose rows the 16-byte copies can stage (bands and row
    stride multiples of 8): two pixel rows per copy instruction."""
    say(f"covariance uint16 copy path n={n} m={m} pad={pad}")
    u = synth.radiance_cube_u16(np.random.default_rng(900 + m), n, m, 6, 1.0)
    ref = oracle.pca(u, 1)
    buf = np.zeros((n, m + pad), dtype=np.uint16)
    buf[:, :m] = u
    Yd = dev(buf)[:, :m] if pad else dev(u)
    for mode in ("f32", "bf16x3", "bf16x4", "fp16x3"):
        C, mean = gpu_cov(pca, Yd, mode)
        err = np.abs(C - ref["C"]).max() / np.abs(ref["C"]).max()
        say(f"  {mode}: {err:.2e}")
        assert err <= COV_TOL[mode], (mode, err)
        assert np.array_equal(C, C.T)
        assert np.abs(mean - ref["mean"]).max() <= 1e-6 * ref["mean"].max()


def test_covariance_centered_flag(pca):
    say("covariance centred input")
    rng = np.random.default_rng(8)
    Yh = synth.mixture_cube(rng, 3000, 40, 4, 1.0, 0.01)
    X = oracle.center(Yh).astype(np.float32)
    refC = X.astype(np.float64).T @ X.astype(np.float64) / (X.shape[0] - 1)
    C, _ = gpu_cov(pca, dev(X), "f32", centered=True)
    assert np.abs(C - refC).max() / np.abs(refC).max() <= COV_TOL["f32"]


def test_center(pca):
    say("pca_center")
    rng = np.random.default_rng(9)
    Yh = synth.mixture_cube(rng, 7777, 45, 4, 1.0, 0.01)
    Yd = dev(Yh)
    mean = torch.empty(45, dtype=torch.float32, device="cuda")
    X = torch.empty(7777, 45, dtype=torch.float32, device="cuda")
    pca.pca_center(Yd, mean, X)
    mu = oracle.band_mean(Yh)
    assert np.abs(host(mean) - mu).max() <= 1e-7 * np.abs(mu).max()
    Xr = oracle.center(Yh, mu)
    assert np.abs(host(X) - Xr).max() <= 1e-6


def jacobi_gpu(P, C, tol=1e-6, max_sweeps=30, fp64_angles=True):
    m = C.shape[0]
    Cd = dev(C.astype(np.float32))
    lam = torch.empty(m, dtype=torch.float32, device="cuda")
    V = torch.empty(m, m, dtype=torch.float32, device="cuda")
    info = P.new_info()
    P.pca_jacobi_eigh(Cd, lam, V, tol, max_sweeps, fp64_angles, info)
    return host(lam), host(V), P.read_info(info)


@pytest.mark.parametrize("m", [2, 3, 4, 7, 16, 33, 64, 127, 128, 224, 256])
def test_jacobi_planted(pca, m):
    say(f"jacobi planted m={m}")
    rng = np.random.default_rng(200 + m)
    lam0 = np.linspace(1.0, 0.05, m)
    A, Q, lam0 = synth.random_symmetric(rng, m, lam0)
    A32 = A.astype(np.float32).astype(np.float64)
    ref_l, ref_V, _ = oracle.jacobi_eigh(A32)
    lam, V, info = jacobi_gpu(pca, A32)
    assert info["converged"] == 1 and info["nonfinite"] == 0, info
    assert eig_err(lam, ref_l) <= EIG_TOL
    r = report(lam, V, None, dict(lam=ref_l, V=ref_V, Q=None), m)
    assert r["angle"] <= ANGLE_TOL, r
    assert r.get("subspace", 0.0) <= SUBSPACE_TOL, r
    assert sign_rule_holds(V, list(range(m)))
    assert np.abs(V.T @ V - np.eye(m)).max() <= 1e-5


def test_jacobi_special_inputs(pca):
    say("jacobi special inputs")
    # Already diagonal: no rotation, zero sweeps, sorted output.
    d = np.array([3.0, -1.0, 7.0, 0.5, 2.0])
    lam, V, info = jacobi_gpu(pca, np.diag(d))
    assert info["sweeps"] == 0 and info["rotations"] == 0
    assert np.array_equal(lam, np.sort(d)[::-1].astype(np.float32))
    assert np.array_equal(np.abs(V), np.eye(5)[:, np.argsort(-d, kind="stable")])
    # A zero row/column (a constant band).
    rng = np.random.default_rng(3)
    A, _, _ = synth.random_symmetric(rng, 9)
    A[4, :] = 0.0
    A[:, 4] = 0.0
    ref_l, _, _ = oracle.jacobi_eigh(A.astype(np.float32).astype(np.float64))
    lam, V, info = jacobi_gpu(pca, A)
    assert info["converged"] == 1 and eig_err(lam, ref_l) <= EIG_TOL
    # Non-finite input is reported and propagates NaN.
    B = np.eye(6)
    B[2, 3] = B[3, 2] = np.nan
    lam, V, info = jacobi_gpu(pca, B)
    assert info["nonfinite"] == 1 and np.all(np.isnan(lam))
    # max_sweeps = 1 stops early and says so.
    A, _, _ = synth.random_symmetric(np.random.default_rng(4), 64)
    lam, V, info = jacobi_gpu(pca, A, tol=1e-12, max_sweeps=1)
    assert info["sweeps"] == 1 and info["converged"] == 0


def run_config(P, name, mode="f32", n_pixels=None, k=None):
    d = synth.make_config(name, n_pixels=n_pixels)
    k = k or d["k"]
    Yh = d.get("Y_u16", d["Y"])
    ref = oracle.pca(Yh, k)
    res = P.run(dev(Yh), k, mode=mode)
    out = report(host(res.eigvals), host(res.V), host(res.Q), ref, k)
    out["info"] = res.read_info()
    out["mean"] = float(np.abs(host(res.mean) - ref["mean"]).max() / np.abs(ref["mean"]).max())
    return out


@pytest.mark.parametrize("name", ["c1", "c2", "c5"])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "bf16x4", "fp16x3"])
def test_end_to_end(pca, name, mode):
    say(f"end-to-end {name} {mode}")
    r = run_config(pca, name, mode)
    say(r)
    assert r["info"]["converged"] == 1
    assert r["eig"] <= EIG_TOL, r
    assert r["angle"] <= ANGLE_TOL, r
    assert r.get("subspace", 0.0) <= SUBSPACE_TOL, r
    assert r["proj"] <= PROJ_TOL, r
    assert r["mean"] <= 1e-6, r


@pytest.mark.parametrize("mode", ["f32", "bf16x3", "bf16x4", "fp16x3"])
def test_end_to_end_224_band_cube(pca, mode):
    say(f"end-to-end c3 full size {mode}")
    r = run_config(pca, "c3", mode)
    say(r)
    assert r["info"]["converged"] == 1
    assert r["eig"] <= EIG_TOL, r
    assert r["angle"] <= ANGLE_TOL, r
    assert r.get("subspace", 0.0) <= SUBSPACE_TOL, r
    assert r["proj"] <= PROJ_TOL, r


def test_projection_direct(pca):
    say("pca_project direct")
    rng = np.random.default_rng(11)
    n, m, k = 999, 37, 21
    Yh = synth.mixture_cube(rng, n, m, 6, 1.0, 0.01)
    mu = oracle.band_mean(Yh)
    Vh = synth.haar_orthogonal(rng, m)
    Q = torch.empty(n, k, dtype=torch.float32, device="cuda")
    pca.pca_project(dev(Yh), dev(mu.astype(np.float32)), dev(Vh.astype(np.float32)), k, Q)
    ref = oracle.project(oracle.center(Yh, mu.astype(np.float32).astype(np.float64)), Vh.astype(np.float32), k)
    assert np.abs(host(Q) - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("n,m,k,u16", [(1000, 224, 10, False), (33, 64, 17, False), (70001, 256, 16, False),
                                       (5003, 224, 10, True), (777, 4, 3, False), (500, 2, 2, False),
                                       (4096, 128, 32, False), (1001, 37, 5, False), (999, 255, 9, False),
                                       (70003, 243, 5, False), (13, 3, 2, False)])
def test_projection_shapes(pca, n, m, k, u16):
    """pca_project on aligned (4 bands a load) and unaligned rows, float32 and
    uint16, pixel counts that are not a multiple of the 32-pixel tile or that
    leave most workgroups without a tile, 1 to 64 K steps (the second band
    half empty for 2 and 4 bands), k up to two 16-column groups, and odd
    band counts up to 255 with ragged last tiles."""
    say(f"pca_project n={n} m={m} k={k} u16={u16}")
    rng = np.random.default_rng(n + m + k)
    if u16:
        Yh = synth.radiance_cube_u16(rng, n, m, 6, 1.0)
    else:
        Yh = synth.mixture_cube(rng, n, m, min(6, m), 1.0, 0.01)
    mu = oracle.band_mean(Yh).astype(np.float32)
    Vh = synth.haar_orthogonal(rng, m).astype(np.float32)
    Q = torch.empty(n, k, dtype=torch.float32, device="cuda")
    pca.pca_project(dev(Yh), dev(mu), dev(Vh), k, Q)
    ref = oracle.project(oracle.center(Yh, mu.astype(np.float64)), Vh, k)
    err = np.abs(host(Q) - ref).max() / np.abs(ref).max()
    say(f"  max rel err {err:.2e}")
    assert err <= 1e-5


def test_deterministic(pca):
    say("determinism")
    d = synth.make_config("c2")
    Yd = dev(d["Y"])
    outs = []
    for _ in range(2):
        r = pca.run(Yd, 8, mode="bf16x3")
        outs.append([host(t).copy() for t in (r.C, r.eigvals, r.V, r.Q)])
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_graph_replay_matches_eager(pca):
    say("hip graph capture")
    d = synth.make_config("c1")
    Yd = dev(d["Y"])
    pipe = pca.PCAPipeline(Yd.shape[0], Yd.shape[1], 3, "bf16x4")
    pipe.forward(Yd)
    eager = [host(t).copy() for t in (pipe.C, pipe.eigvals, pipe.V, pipe.Q)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        pipe.forward(Yd)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            pipe.forward(Yd)
    torch.cuda.synchronize()
    for _ in range(3):
        for t in (pipe.C, pipe.eigvals, pipe.V, pipe.Q):
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, t in zip(eager, (pipe.C, pipe.eigvals, pipe.V, pipe.Q)):
            assert np.array_equal(a, host(t))


def test_argument_errors(pca):
    say("argument errors")
    Y = torch.zeros(10, 4, device="cuda")
    C = torch.empty(4, 4, device="cuda")
    with pytest.raises(pca.PCAError):
        pca.pca_covariance(Y[:1], C)           # one pixel
    with pytest.raises(pca.PCAError):
        pca.pca_project(Y, None, C, 5, torch.empty(10, 5, device="cuda"))   # k > bands
    small = pca.workspace(256)
    with pytest.raises(pca.PCAError):
        pca.pca_covariance(torch.zeros(100000, 64, device="cuda"), torch.empty(64, 64, device="cuda"), ws=small)
