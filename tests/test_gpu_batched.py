"""Batched form (pca_batched through BatchedPCA): every cube of a batch of
uneven pixel and band counts against the FP64 oracle, against the
single-cube GPU path, under graph capture and under each tile shape the
autotuner may pick."""

from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import eig_err, report, SUBSPACE_TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EIG_TOL = 1e-5
ANGLE_TOL = 1e-4
PROJ_TOL = 1e-4
# Batched vs single-cube GPU results: the same kernels with a different pixel
# chunking (float32 partial sums over other pixel sets), so they agree to
# float32 rounding of the covariance (~1e-6 of lambda_max), not bitwise.
SAME_TOL = 2e-6


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


# (pixels, bands, k): odd and even band counts on both sides of 128, a
# two-band cube, fewer pixels than bands (rank-deficient covariance), a
# pixel count that is not a multiple of the 32-pixel stage.
SMALL = [(700, 37, 3), (4096, 64, 5), (1500, 2, 1), (3000, 129, 7), (2000, 255, 5), (64, 100, 4),
         (20001, 224, 10), (5000, 256, 6)]


def small_batch(dtype=np.float32):
    cubes = []
    for i, (n, m, k) in enumerate(SMALL):
        rng = np.random.default_rng(700 + i)
        if dtype == np.uint16:
            cubes.append(synth.radiance_cube_u16(rng, n, m, 6, 1.0))
        else:
            cubes.append(synth.mixture_cube(rng, n, m, min(8, max(2, m // 4)), 1.0, 0.01))
    return cubes, [k for (_, _, k) in SMALL]


def check_against_oracle(P, b, cubes, ks, label):
    for i, (Y, k) in enumerate(zip(cubes, ks)):
        info = P.read_info(b.info[i])
        ref = oracle.pca(Y, k)
        r = report(host(b.eigvals[i]), host(b.V[i]), host(b.Q[i]), ref, k)
        mu_err = float(np.abs(host(b.mean[i]) - ref["mean"]).max() / max(1.0, np.abs(ref["mean"]).max()))
        say(f"{label} cube {i} {Y.shape} k={k}: eig {r['eig']:.2e} angle {r['angle']:.2e} proj {r['proj']:.2e} "
            f"mean {mu_err:.1e} sweeps {info['sweeps']}")
        assert info["converged"] == 1
        assert r["eig"] <= EIG_TOL, (i, r)
        assert r["angle"] <= ANGLE_TOL, (i, r)
        assert r["proj"] <= PROJ_TOL, (i, r)
        assert r.get("subspace", 0.0) <= SUBSPACE_TOL, (i, r)
        assert mu_err <= 1e-6


@pytest.mark.parametrize("mode", ["f32", "bf16x3", "fp16x3"])
def test_batched_matches_oracle(pca, mode):
    cubes, ks = small_batch()
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, mode)
    b.run()
    check_against_oracle(pca, b, cubes, ks, f"batched {mode}")


@pytest.mark.parametrize("dtype,mode", [(np.float32, "f32"), (np.float32, "bf16x3"), (np.uint16, "fp16x3"),
                                        (np.uint16, "bf16x4")])
def test_batched_band_sequential(pca, dtype, mode):
    """Band-sequential cubes ([bands, pixels]; one with a padded band stride)
    through the batched form, against the oracle and against the same cubes
    band-interleaved through the batched form."""
    cubes, ks = small_batch(dtype)
    bsq = []
    for i, Y in enumerate(cubes):
        if i == 1:
            buf = np.zeros((Y.shape[1], Y.shape[0] + 5), dtype=Y.dtype)
            buf[:, :Y.shape[0]] = Y.T
            bsq.append(dev(buf)[:, :Y.shape[0]])
        else:
            bsq.append(dev(Y.T))
    b = pca.BatchedPCA(bsq, ks, mode, layout="bsq")
    b.run()
    check_against_oracle(pca, b, cubes, ks, f"batched bsq {np.dtype(dtype).name} {mode}")
    bb = pca.BatchedPCA([dev(Y) for Y in cubes], ks, mode)
    bb.run()
    for i in range(len(cubes)):
        d = np.abs(host(b.eigvals[i]) - host(bb.eigvals[i])).max() / abs(host(bb.eigvals[i])).max()
        assert d <= 1e-5, (i, d)


def test_batched_uint16(pca):
    cubes, ks = small_batch(np.uint16)
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, "bf16x3")
    b.run()
    check_against_oracle(pca, b, cubes, ks, "batched u16")


def test_batched_matches_single_cube_path(pca):
    cubes, ks = small_batch()
    Yd = [dev(Y) for Y in cubes]
    b = pca.BatchedPCA(Yd, ks, "f32")
    b.run()
    for i, (Y, k) in enumerate(zip(Yd, ks)):
        s = pca.run(Y, k, "f32")
        lam_s, lam_b = host(s.eigvals), host(b.eigvals[i])
        err = eig_err(lam_b, lam_s.astype(np.float64))
        say(f"cube {i}: batched vs single eig {err:.2e}")
        assert err <= SAME_TOL


def test_batched_workload_64_cubes(pca):
    """The 64-cube workload (square sides 64..512 capped at 256 here to keep
    the host-side generation and the oracle short; band counts 64..256
    unchanged): every cube converges with orthonormal eigenvectors, and a
    sample of cubes matches the oracle."""
    cubes = synth.make_batch(64, 4000, max_side=256)
    ks = [5] * len(cubes)
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, "bf16x3")
    b.run()
    for i in range(len(cubes)):
        info = pca.read_info(b.info[i])
        assert info["converged"] == 1, (i, info)
        V = host(b.V[i]).astype(np.float64)
        assert np.abs(V.T @ V - np.eye(V.shape[0])).max() <= 1e-4, i
    bands = [Y.shape[1] for Y in cubes]
    pix = [Y.shape[0] for Y in cubes]
    sample = sorted({int(np.argmax(bands)), int(np.argmin(bands)), int(np.argmax(pix)), int(np.argmin(pix))})
    check_against_oracle(pca, _Sub(b, sample), [cubes[i] for i in sample], [ks[i] for i in sample], "c4")


def test_batched_full_workload_f32(pca):
    """The 64-cube workload at its full sizes (square sides 64..512, 64..256
    bands, k = 5) in float32: every cube against the FP64 oracle
    (eigenvalues, well-separated eigenvectors, projections, leading
    subspace)."""
    cubes = synth.make_batch(64, 4000)
    ks = [5] * len(cubes)
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, "f32")
    b.run()
    check_against_oracle(pca, b, cubes, ks, "c4 full f32")


class _Sub:
    """View of some cubes of a BatchedPCA (for check_against_oracle)."""

    def __init__(self, b, idx):
        self.info = [b.info[i] for i in idx]
        self.eigvals = [b.eigvals[i] for i in idx]
        self.V = [b.V[i] for i in idx]
        self.Q = [b.Q[i] for i in idx]
        self.mean = [b.mean[i] for i in idx]


def _snapshot(b):
    return [host(t).copy() for t in b.eigvals + b.V + b.Q + b.mean]


def test_batched_graph_replay(pca):
    """A captured pca_batched call replayed several times, with eager work in
    between, reproduces the eager outputs bitwise."""
    cubes, ks = small_batch()
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, "bf16x3")
    b.run()
    ref = _snapshot(b)
    g = b.capture()
    for rep in range(3):
        for t in b.eigvals + b.V + b.Q + b.mean:
            t.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(b)
        assert all(np.array_equal(a, c) for a, c in zip(ref, got)), rep


@pytest.mark.parametrize("tuning", [(2048, 4), (4096, 8), (16384, 32), (32, 1)])
def test_batched_tile_shapes(pca, tuning):
    """Every tile shape the autotuner may choose gives oracle-matching,
    deterministic results."""
    cubes, ks = small_batch()
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, "f32", tuning=tuning)
    b.run()
    first = _snapshot(b)
    b.run()
    assert all(np.array_equal(a, c) for a, c in zip(first, _snapshot(b)))
    check_against_oracle(pca, b, cubes, ks, f"tuning {tuning}")


def test_autotune(pca, tmp_path, monkeypatch):
    from paper_2403_18321_amd import autotune
    monkeypatch.setenv("PCA_TUNING_CACHE", str(tmp_path / "tuning.json"))
    cubes, ks = small_batch()
    b = pca.BatchedPCA([dev(Y) for Y in cubes], ks, "bf16x3")
    best, times = autotune.tune(b, reps=2)
    say(f"autotune: {best}")
    assert best["cov_chunk"] in autotune.COV_CHUNKS and best["proj_tiles"] in autotune.PROJ_TILES
    assert len(times) == len(autotune.COV_CHUNKS) + len(autotune.PROJ_TILES)
    assert os.path.exists(tmp_path / "tuning.json")
    again, times2 = autotune.tune(b)
    assert again == best and times2 == {}
    b.run()
    check_against_oracle(pca, b, cubes, ks, "autotuned")


def test_batched_argument_errors(pca):
    cubes, ks = small_batch()
    Yd = [dev(Y) for Y in cubes[:2]]
    with pytest.raises(ValueError):
        pca.BatchedPCA([], [])
    with pytest.raises(pca.PCAError):
        pca.BatchedPCA(Yd, [1, 1000])          # k > bands
    with pytest.raises(pca.PCAError):
        pca.BatchedPCA(Yd, [1, 1], tuning=(100, 4))   # chunk not a multiple of 32


def test_batched_lanes_bitwise(pca):
    """Splitting the batch into lanes (sub-batches by band count, each on its
    own stream) changes no cube's result: every cube's work items are the
    same whatever else is in its sub-batch. Also under graph capture."""
    cubes, ks = small_batch()
    Yd = [dev(Y) for Y in cubes]
    one = pca.BatchedPCA(Yd, ks, "bf16x3")
    one.run()
    ref = _snapshot(one)
    three = pca.BatchedPCA(Yd, ks, "bf16x3", lanes=3)
    assert len(three.groups) == 3 and sorted(i for g in three.groups for i in g) == list(range(len(cubes)))
    three.run()
    assert all(np.array_equal(a, c) for a, c in zip(ref, _snapshot(three)))
    g = three.capture()
    for rep in range(2):
        for t in three.eigvals + three.V + three.Q + three.mean:
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert all(np.array_equal(a, c) for a, c in zip(ref, _snapshot(three))), rep
