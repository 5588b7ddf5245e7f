"""The split-float16 covariance form (PCA_COV_FP16X3) on inputs that exercise
its per-band power-of-two scales: bands of very different magnitudes, and a
value beyond the float16 range after scaling, which must surface as a
non-finite covariance rather than a wrong one."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# Per entry, relative to sqrt(C_ii C_jj): each product x_i x_j is off by at
# most 3 * 2^-22 of |x_i x_j| (22-bit hi/lo pair of the scaled value, lo*lo
# dropped), and Cauchy-Schwarz bounds the sum by sqrt(C_ii C_jj) (N - 1) / N;
# float32 accumulation adds the bound the float32 form is held to.
ENTRY_TOL = 3e-6


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


def covariance(P, Y, mode):
    n, m = Y.shape
    C = torch.empty(m, m, dtype=torch.float32, device="cuda")
    mean = torch.empty(m, dtype=torch.float32, device="cuda")
    P.pca_covariance(Y, C, mean, P.COV_MODES[mode], False)
    return host(C).astype(np.float64), host(mean)


@pytest.mark.parametrize("m,ld", [(48, 48), (45, 45), (64, 70)])
def test_bands_of_different_magnitude(pca, m, ld):
    """Bands scaled by 10^-3 .. 10^3: every entry within ENTRY_TOL of its own
    scale, which a single (not per-band) float16 scale could not reach for
    the small bands."""
    n = 30000
    Y = synth.mixture_cube(np.random.default_rng(77 + m), n, m, 5, 1.0, 0.01)
    Y = (Y * (10.0 ** ((np.arange(m) % 7) - 3))[None, :]).astype(np.float32)
    ref = oracle.pca(Y, 3)
    buf = np.zeros((n, ld), dtype=np.float32)
    buf[:, :m] = Y
    Yd = torch.from_numpy(buf).cuda()[:, :m]
    d = np.sqrt(np.diag(ref["C"]))
    for mode in ("fp16x3", "f32"):
        C, mean = covariance(pca, Yd, mode)
        rel = np.abs(C - ref["C"]) / np.outer(d, d)
        say(f"m={m} ld={ld} {mode}: max entry error {rel.max():.2e}")
        assert rel.max() <= ENTRY_TOL, (mode, rel.max())
        assert np.all(np.abs(mean - ref["mean"]) <= 1e-6 * np.abs(ref["mean"]) + 1e-12)
    res = pca.run(Yd, 3, mode="fp16x3")
    r = report(host(res.eigvals), host(res.V), host(res.Q), ref, 3)
    say(f"  pipeline fp16x3: {r}")
    assert res.read_info()["converged"] == 1 and r["eig"] <= 1e-5, r


@pytest.mark.parametrize("layout", ["bip", "bsq"])
def test_overflow_is_reported(pca, layout):
    """One value far outside its band's sampled spread (at a pixel that the
    shift sample skips): the float16 split overflows, the covariance and the
    eigenpairs come out non-finite and the Jacobi call reports it; the float32
    form on the same cube is finite and matches the oracle."""
    n, m = 20000, 40
    Y = synth.mixture_cube(np.random.default_rng(5), n, m, 4, 1.0, 0.01)
    Y[1, 3] = 1.0e7
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    if layout == "bsq":
        Yd = Yd.t().contiguous()
    res = pca.run(Yd, 3, mode="fp16x3", layout=layout)
    info = res.read_info()
    say(f"{layout} fp16x3: {info}")
    assert info["nonfinite"] == 1, info
    assert not np.all(np.isfinite(host(res.C)))
    assert np.all(np.isnan(host(res.eigvals)))
    res = pca.run(Yd, 3, mode="f32", layout=layout)
    ref = oracle.pca(Y, 3)
    r = report(host(res.eigvals), host(res.V), host(res.Q), ref, 3)
    assert res.read_info()["nonfinite"] == 0 and r["eig"] <= 1e-5, r
