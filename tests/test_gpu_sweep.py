"""The paper's synthetic sweep shapes (Section 6: 100^2 .. 500^2 pixels x 50
bands, 300^2 pixels x 20 .. 200 bands) on this repository's own 70 dB SNR
mixtures, through the whole pipeline against the FP64 oracle."""

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


@pytest.mark.parametrize("i", range(len(synth.SWEEP_SHAPES)))
@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_sweep_shape(pca, i, mode):
    n, m = synth.SWEEP_SHAPES[i]
    k = 3
    Yh = synth.snr_mixture_cube(np.random.default_rng(5000 + i), n, m)
    ref = oracle.pca(Yh, k)
    res = pca.run(torch.from_numpy(Yh).cuda(), k, mode=mode)
    torch.cuda.synchronize()
    r = report(res.eigvals.cpu().numpy(), res.V.cpu().numpy(), res.Q.cpu().numpy(), ref, k)
    info = res.read_info()
    say(f"{n} px x {m} bands {mode}: {r} sweeps {info['sweeps']}")
    assert info["converged"] == 1
    assert r["eig"] <= 1e-5
    assert r["angle"] <= 1e-4 and r["proj"] <= 1e-4
    assert r.get("subspace", 0.0) <= SUBSPACE_TOL, r
