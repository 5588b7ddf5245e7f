"""Band-sequential (BSQ) cubes, the layout of the paper's GPU design
([bands][pixels], a band's pixels contiguous): centring, covariance and
projection through the C ABI against the FP64 oracle on the same values, and
against the band-interleaved path on the transposed copy of the same cube."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import report, SUBSPACE_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EIG_TOL = 1e-5
ANGLE_TOL = 1e-4
PROJ_TOL = 1e-4
COV_TOL = {"f32": 2e-6, "bf16x4": 2e-6, "bf16x3": 3e-5, "fp16x3": 3e-6}


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


def bsq(Y, pad=0):
    """Device copy of a [pixels, bands] host cube as [bands, pixels], each band
    row padded by `pad` elements (the band stride is pixels + pad)."""
    n, m = Y.shape
    buf = np.zeros((m, n + pad), dtype=Y.dtype)
    buf[:, :n] = Y.T
    t = torch.from_numpy(buf).cuda()
    return t[:, :n] if pad else t


def cov(P, Y, mode, layout, centered=False):
    m = Y.shape[0] if layout == "bsq" else Y.shape[1]
    C = torch.empty(m, m, dtype=torch.float32, device="cuda")
    mean = torch.empty(m, dtype=torch.float32, device="cuda")
    P.pca_covariance(Y, C, None if centered else mean, P.COV_MODES[mode], centered, layout=layout)
    return host(C), host(mean)


# (pixels, bands, band-stride padding): ragged pixel counts (not a multiple of
# the 32-pixel stage), band counts on both sides of the 32-band blocks, the
# band limit (256, where the float32 products take several passes), padding.
# Pixel counts and band strides that are multiples of 4 take the LDS-copy
# kernel in the split forms (one stage, ragged chunks, every
# band count class), the others the register-staged one.
SHAPES = [(1000, 2, 0), (3001, 37, 5), (4096, 64, 0), (2500, 129, 3), (20001, 224, 0), (5000, 255, 1),
          (3333, 256, 0), (4, 8, 0), (2016, 64, 0), (20000, 224, 0), (5000, 255, 4), (2048, 256, 0), (9996, 33, 8)]


@pytest.mark.parametrize("n,m,pad", SHAPES)
def test_bsq_covariance(pca, n, m, pad):
    say(f"bsq covariance n={n} m={m} pad={pad}")
    Yh = synth.mixture_cube(np.random.default_rng(300 + m), n, m, min(8, max(2, m // 4)), 1.0, 0.01)
    ref = oracle.pca(Yh, 1)
    Yb = bsq(Yh, pad)
    Yi = torch.from_numpy(Yh).cuda()
    scale = np.abs(ref["C"]).max()
    for mode in ("f32", "bf16x3", "bf16x4", "fp16x3"):
        C, mean = cov(pca, Yb, mode, "bsq")
        Ci, _ = cov(pca, Yi, mode, "bip")
        err = np.abs(C - ref["C"]).max() / scale
        say(f"  {mode}: vs oracle {err:.2e}, vs bip {np.abs(C - Ci).max() / scale:.2e}")
        assert err <= COV_TOL[mode], (mode, err)
        assert np.array_equal(C, C.T)
        assert np.abs(mean - ref["mean"]).max() <= 1e-6 * np.abs(ref["mean"]).max()


def test_bsq_uint16_and_centered(pca):
    say("bsq uint16, centred flag")
    n, m = 7000, 96
    u = synth.radiance_cube_u16(np.random.default_rng(31), n, m, 6, 1.0)
    ref = oracle.pca(u, 1)
    # band stride 7002: register-staged; 7008 (a multiple of 8 uint16): LDS
    # copies in the split forms
    for pad in (2, 8):
        Yb = bsq(u, pad)
        for mode in ("f32", "bf16x3", "bf16x4", "fp16x3"):
            C, mean = cov(pca, Yb, mode, "bsq")
            err = np.abs(C - ref["C"]).max() / np.abs(ref["C"]).max()
            say(f"  pad {pad} {mode}: {err:.2e}")
            assert err <= COV_TOL[mode], (pad, mode, err)
            assert np.abs(mean - ref["mean"]).max() <= 1e-6 * np.abs(ref["mean"]).max()
    # centred input: C = Y^T Y / (N - 1)
    X = (u.astype(np.float64) - u.astype(np.float64).mean(0)).astype(np.float32)
    Cc, _ = cov(pca, bsq(X), "f32", "bsq", centered=True)
    Xd = X.astype(np.float64)
    Cref = Xd.T @ Xd / (n - 1)
    assert np.abs(Cc - Cref).max() / np.abs(Cref).max() <= 2e-6


@pytest.mark.parametrize("n,m,pad", [(3001, 37, 5), (20001, 224, 0)])
def test_bsq_center(pca, n, m, pad):
    Yh = synth.mixture_cube(np.random.default_rng(400 + m), n, m, 5, 1.0, 0.01)
    Yb = bsq(Yh, pad)
    mean = torch.empty(m, dtype=torch.float32, device="cuda")
    X = torch.empty(m, n + 3, dtype=torch.float32, device="cuda")[:, :n]
    pca.pca_center(Yb, mean, X, layout="bsq")
    mu = Yh.astype(np.float64).mean(0)
    assert np.abs(host(mean) - mu).max() <= 1e-6 * np.abs(mu).max()
    Xref = (Yh.astype(np.float64) - mu).T
    assert np.abs(host(X) - Xref).max() <= 1e-6 * np.abs(Yh).max()


@pytest.mark.parametrize("dtype", ["f32", "u16"])
def test_bsq_end_to_end(pca, dtype):
    """run(layout="bsq") against the oracle, and the projection against the
    band-interleaved projection with the same eigenvectors."""
    n, m, k = 30000, 128, 8
    rng = np.random.default_rng(77)
    Yh = synth.radiance_cube_u16(rng, n, m, 10, 0.5) if dtype == "u16" else synth.mixture_cube(rng, n, m, 10, 0.5, 0.005)
    ref = oracle.pca(Yh, k)
    Yb = bsq(Yh)
    for mode in ("f32", "bf16x4"):
        r = pca.run(Yb, k, mode, layout="bsq")
        rep = report(host(r.eigvals), host(r.V), host(r.Q), ref, k)
        say(f"bsq {dtype} {mode}: eig {rep['eig']:.2e} angle {rep['angle']:.2e} proj {rep['proj']:.2e}")
        assert pca.read_info(r.info)["converged"] == 1
        assert rep["eig"] <= EIG_TOL and rep["angle"] <= ANGLE_TOL and rep["proj"] <= PROJ_TOL
        assert rep.get("subspace", 0.0) <= SUBSPACE_TOL, rep
        Qi = torch.empty(n, k, dtype=torch.float32, device="cuda")
        pca.pca_project(torch.from_numpy(Yh).cuda(), r.mean, r.V, k, Qi)
        Qb = host(r.Q)
        assert np.abs(Qb - host(Qi)).max() <= 1e-5 * np.abs(Qb).max()


def test_bsq_argument_errors(pca):
    Yb = bsq(synth.mixture_cube(np.random.default_rng(5), 500, 16, 3, 1.0, 0.01))
    C = torch.empty(16, 16, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        pca.pca_covariance(Yb, C, layout="bsx")
    # a band stride shorter than the pixel count
    lib = pca.library()
    import ctypes
    ws = pca.workspace(pca.pca_workspace_size(pca.PCA_OP_COVARIANCE, 500, 16), Yb.device)
    st = lib.pca_covariance(ctypes.c_void_p(Yb.data_ptr()), pca.PCA_IN_F32_BSQ, 500, 16, 499, 0, None, 0,
                            ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == 1
