"""The whole pipeline (through the C ABI) on cubes with a defective detector
column, a constant band and a non-finite pixel, against the FP64 oracle."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from parity_utils import SUBSPACE_TOL, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EIG_TOL = 1e-5
ANGLE_TOL = 1e-4
PROJ_TOL = 1e-4
# Covariance entries relative to max |C|, worst case over the data. A
# bfloat16 hi/lo pair holds x to |x - hi - lo| <= 2^-16 |x| (unit roundoff
# 2^-8 twice), so each product x_i x_j is off by at most 2 * 2^-16 of
# |x_i x_j| (bf16x4), plus the dropped lo_i lo_j <= 2^-16 |x_i x_j| (bf16x3);
# summed over pixels and bounded by Cauchy-Schwarz, |dC_ij| <= that fraction
# of sqrt(C_ii C_jj) <= max |C|. On cubes with many identical outliers the
# rounding errors add up coherently and approach these bounds (random data
# stays near float32 rounding, the bound of the covariance shape tests).
# The float16 split: 3 * 2^-22 of |x_i x_j| per product (22-bit pair, lo*lo
# dropped) on top of the float32 accumulation bound.
COV_TOL = {"f32": 2e-6, "bf16x4": 3.1e-5, "bf16x3": 4.7e-5, "fp16x3": 3e-6}


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


_CACHE = {}


def column_cube(kind, value):
    """A 1024-pixel-wide scene whose image column 0 is dead (0) or hot (5 x
    the cube's maximum; 65535 for uint16): the covariance chunks of these
    sizes (2048 float32 pixels of 128 bands; 1024 uint16 pixels of 224
    bands) all start on that column."""
    key = (kind, value)
    if key not in _CACHE:
        if kind == "f32":
            Y = synth.make_config("c2", n_pixels=512 * 1024)["Y"].copy()
            Y[::1024, :] = 0.0 if value == "dead" else 5.0 * float(Y.max())
        else:
            Y = synth.make_config("c3", n_pixels=256 * 1024)["Y_u16"].copy()
            Y[::1024, :] = 0 if value == "dead" else 65535
        _CACHE[key] = (Y, oracle.pca(Y, 10 if kind == "u16" else 8))
    return _CACHE[key]


def check(P, Y, ref, k, mode, layout="bip", coherent_outliers=False):
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    if layout == "bsq":
        Yd = Yd.t().contiguous()
    res = P.run(Yd, k, mode=mode, layout=layout)
    C = host(res.C).astype(np.float64)
    cov = float(np.abs(C - ref["C"]).max() / np.abs(ref["C"]).max())
    r = report(host(res.eigvals), host(res.V), host(res.Q), ref, k)
    info = res.read_info()
    say(f"  {mode} {layout}: cov {cov:.2e} {r} sweeps {info['sweeps']}")
    assert info["converged"] == 1 and info["nonfinite"] == 0, info
    assert cov <= COV_TOL[mode], cov
    assert r["eig"] <= EIG_TOL, r
    if mode == "bf16x3" and coherent_outliers:
        # bf16x3 leaves out every lo_i lo_j product, a bias that many identical
        # outlier pixels add up coherently; the eigenvalue bound (the precision
        # form's requirement) and the covariance bound above still hold, and
        # the eigenvector and projection errors are reported, not bounded.
        return
    assert r["angle"] <= ANGLE_TOL and r["proj"] <= PROJ_TOL, r
    assert r.get("subspace", 0.0) <= SUBSPACE_TOL, r


@pytest.mark.parametrize("value", ["dead", "hot"])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "bf16x4", "fp16x3"])
def test_defective_column_f32(pca, value, mode):
    say(f"float32 cube, {value} column 0, {mode}")
    Y, ref = column_cube("f32", value)
    check(pca, Y, ref, 8, mode, coherent_outliers=value == "hot")
    if mode in ("bf16x3", "fp16x3"):
        check(pca, Y, ref, 8, mode, layout="bsq", coherent_outliers=value == "hot")


@pytest.mark.parametrize("value", ["dead", "hot"])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "fp16x3"])
def test_defective_column_u16(pca, value, mode):
    say(f"uint16 cube, {value} column 0, {mode}")
    Y, ref = column_cube("u16", value)
    check(pca, Y, ref, 10, mode, coherent_outliers=value == "hot")
    if mode in ("bf16x3", "fp16x3"):
        check(pca, Y, ref, 10, mode, layout="bsq", coherent_outliers=value == "hot")


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_constant_band(pca, mode):
    """A band that holds one value everywhere: its row and column of C are
    zero and one eigenvalue is zero; the other eigenpairs as the oracle's."""
    say(f"constant band {mode}")
    Y = synth.make_config("c1")["Y"].copy()
    Y[:, 5] = np.float32(0.37)
    ref = oracle.pca(Y, 3)
    check(pca, Y, ref, 3, mode)


def test_nonfinite_pixel(pca):
    """A NaN in one pixel: the call reports non-finite input and every
    eigenvalue, eigenvector and projection is NaN; the next cube through
    the same pipeline is correct again."""
    say("NaN pixel")
    Y = synth.make_config("c1")["Y"].copy()
    n, m = Y.shape
    P = pca.PCAPipeline(n, m, 3, "f32")
    bad = Y.copy()
    bad[17, 3] = np.nan
    res = P.forward(torch.from_numpy(bad).cuda())
    info = res.read_info()
    assert info["nonfinite"] == 1, info
    assert np.all(np.isnan(host(res.eigvals))) and np.all(np.isnan(host(res.V))) and np.all(np.isnan(host(res.Q)))
    res = P.forward(torch.from_numpy(Y).cuda())
    r = report(host(res.eigvals), host(res.V), host(res.Q), oracle.pca(Y, 3), 3)
    assert res.read_info()["nonfinite"] == 0
    assert r["eig"] <= EIG_TOL and r["angle"] <= ANGLE_TOL and r["proj"] <= PROJ_TOL, r
