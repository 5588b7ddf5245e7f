"""Seeded generators for the synthetic workloads.

The paper evaluates on synthetic cubes built by linear mixing of library
spectral signatures plus Gaussian noise (Section 6, the spatial and spectral
sweeps) and on AVIRIS scenes (Table 1). Neither the signature library nor the
scenes are available, so these generators stand in for them: endmember spectra
are sums of Gaussians over the band index, abundances are Dirichlet draws, and
noise is Gaussian (float cubes) or Poisson-like (uint16 radiance cubes). Only
shapes and value statistics are borrowed; no data item of any suite is
reproduced.

Every generator takes a ``numpy.random.Generator`` (PCG64 through
``numpy.random.default_rng(seed)``) and draws in a fixed order and fixed chunk
size, so a seed reproduces a cube bit for bit on any machine.
"""

from __future__ import annotations

import numpy as np

# Pixels generated per chunk (fixes the order of random draws independently of
# the machine, and bounds host memory for the 1M-pixel cube).
_CHUNK = 1 << 17

# Workload table: shapes, mixture statistics, number of kept components and
# seeds. "kind" selects the generator.
CONFIGS = {
    # 64x64 pixels x 32 bands, 5 endmembers, Dirichlet(1), noise sigma 0.01.
    "c1": dict(kind="mixture", h=64, w=64, bands=32, r=5, alpha=1.0,
               sigma=0.01, k=3, seed=1001),
    # 512x614 pixels x 128 bands, 10 endmembers, Dirichlet(0.5), sigma 0.005.
    "c2": dict(kind="mixture", h=512, w=614, bands=128, r=10, alpha=0.5,
               sigma=0.005, k=8, seed=1002),
    # 1024x1024 pixels x 224 bands, uint16 radiance with Poisson-like noise.
    "c3": dict(kind="radiance_u16", h=1024, w=1024, bands=224, r=12,
               alpha=1.0, k=10, seed=1003),
    # 64 cubes of uneven size (shapes from batch_shapes), k = 5.
    "c4": dict(kind="batch", n_cubes=64, k=5, seed=4000),
    # 256x256 pixels x 128 bands with a planted covariance spectrum.
    "c5": dict(kind="planted", h=256, w=256, bands=128, k=8, seed=1005),
}


def endmember_spectra(rng: np.random.Generator, r: int, bands: int) -> np.ndarray:
    """r spectra over ``bands`` bands, each a sum of 3 Gaussian bumps.

    Bump centres are uniform over the band index, widths uniform in
    [bands/32, bands/6], amplitudes uniform in [0.2, 1]; each spectrum is then
    min-max scaled to [0, 1]. Returns float64 (r, bands).
    """
    b = np.arange(bands, dtype=np.float64)
    out = np.empty((r, bands), dtype=np.float64)
    for e in range(r):
        c = rng.uniform(0.0, bands, size=3)
        w = rng.uniform(bands / 32.0, bands / 6.0, size=3)
        a = rng.uniform(0.2, 1.0, size=3)
        s = np.zeros(bands)
        for g in range(3):
            s += a[g] * np.exp(-((b - c[g]) ** 2) / (2.0 * w[g] ** 2))
        lo, hi = s.min(), s.max()
        out[e] = (s - lo) / (hi - lo) if hi > lo else np.zeros(bands)
    return out


def mixture_cube(rng, n_pixels: int, bands: int, r: int, alpha: float,
                 sigma: float, dtype=np.float32) -> np.ndarray:
    """Linear-mixing cube Y = A E + noise, band-interleaved-by-pixel [N][M].

    A holds Dirichlet(alpha) abundances per pixel, E the endmember spectra,
    noise is N(0, sigma^2) per entry.
    """
    E = endmember_spectra(rng, r, bands)
    Y = np.empty((n_pixels, bands), dtype=dtype)
    for p0 in range(0, n_pixels, _CHUNK):
        n = min(_CHUNK, n_pixels - p0)
        A = rng.dirichlet(np.full(r, alpha), size=n)
        Y[p0:p0 + n] = A @ E + sigma * rng.standard_normal((n, bands))
    return Y


def snr_mixture_cube(rng, n_pixels: int, bands: int, r: int = 10, snr_db: float = 70.0,
                     dtype=np.float32) -> np.ndarray:
    """Linear-mixing cube (Dirichlet(1) abundances of r endmember spectra)
    with white Gaussian noise at a given signal-to-noise ratio: the noise
    standard deviation is the root-mean-square of the noise-free cube times
    10^(-snr_db / 20) (the shape of the paper's synthetic sweeps, Section 6,
    on this module's own spectra)."""
    Y = mixture_cube(rng, n_pixels, bands, r, 1.0, 0.0, dtype=np.float64)
    sigma = float(np.sqrt(np.mean(Y * Y))) * 10.0 ** (-snr_db / 20.0)
    for p0 in range(0, n_pixels, _CHUNK):
        n = min(_CHUNK, n_pixels - p0)
        Y[p0:p0 + n] += sigma * rng.standard_normal((n, bands))
    return Y.astype(dtype)


# The paper's synthetic sweeps (Section 6): square scenes of 100^2 .. 500^2
# pixels with 50 bands, and 300^2 pixels with 20, 30, 100 and 200 bands.
SWEEP_SHAPES = [(s * s, 50) for s in (100, 200, 300, 400, 500)] + [(300 * 300, b) for b in (20, 30, 100, 200)]


def radiance_cube_u16(rng, n_pixels: int, bands: int, r: int, alpha: float,
                      offset: float = 500.0, scale: float = 64000.0) -> np.ndarray:
    """uint16 radiance cube: offset + scale * (A E), with Poisson-like noise.

    The noise is the Gaussian approximation of a Poisson count (variance equal
    to the mean, which is >= 500 here), rounded to the nearest integer and
    clipped to [0, 65535].
    """
    E = endmember_spectra(rng, r, bands)
    Y = np.empty((n_pixels, bands), dtype=np.uint16)
    for p0 in range(0, n_pixels, _CHUNK):
        n = min(_CHUNK, n_pixels - p0)
        A = rng.dirichlet(np.full(r, alpha), size=n)
        lam = offset + scale * (A @ E)
        y = np.rint(lam + np.sqrt(lam) * rng.standard_normal((n, bands)))
        Y[p0:p0 + n] = np.clip(y, 0, 65535).astype(np.uint16)
    return Y


def haar_orthogonal(rng, m: int) -> np.ndarray:
    """Haar-distributed m x m orthogonal matrix (QR of a Gaussian, sign-fixed)."""
    G = rng.standard_normal((m, m))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


def planted_spectrum(bands: int, stress: bool = False) -> np.ndarray:
    """Eigenvalues for the planted cube.

    Top 8: 1.0, 0.9, ..., 0.3 (gaps 0.1 lambda_max), or with ``stress`` the
    values 1 - 1e-3 (i - 1), whose gaps are exactly 1e-3 lambda_max.
    The rest: 0.2 * 0.9^(i-9) for i >= 9 (1-based).
    """
    lam = np.empty(bands)
    top = min(8, bands)
    if stress:
        lam[:top] = 1.0 - 1e-3 * np.arange(top)
    else:
        lam[:top] = 1.0 - 0.1 * np.arange(top)
    if bands > 8:
        lam[8:] = 0.2 * 0.9 ** np.arange(bands - 8)
    return lam


def planted_cube(rng, n_pixels: int, bands: int, lam=None, stress: bool = False,
                 mu_range=(0.2, 0.8)):
    """Cube whose sample covariance (normalised by N-1) is exactly Q diag(lam) Q^T.

    Z has orthonormal columns orthogonal to the all-ones vector (thin QR of
    [1, G] with the first column dropped), scaled by sqrt(N-1); the cube is
    X = Z diag(sqrt(lam)) Q^T + 1 mu^T with Q Haar-distributed and mu uniform.
    Returns (X float64 [N][M], Q, lam, mu); cast X to float32 for the GPU.
    """
    if lam is None:
        lam = planted_spectrum(bands, stress=stress)
    lam = np.asarray(lam, dtype=np.float64)
    Q = haar_orthogonal(rng, bands)
    H = np.empty((n_pixels, bands + 1))
    H[:, 0] = 1.0
    H[:, 1:] = rng.standard_normal((n_pixels, bands))
    Qz, _ = np.linalg.qr(H)
    Z = Qz[:, 1:] * np.sqrt(n_pixels - 1.0)
    mu = rng.uniform(mu_range[0], mu_range[1], size=bands)
    X = (Z * np.sqrt(lam)) @ Q.T + mu
    return X, Q, lam, mu


def random_symmetric(rng, m: int, lam=None) -> tuple:
    """Symmetric m x m matrix Q diag(lam) Q^T with Haar Q. Returns (A, Q, lam)."""
    if lam is None:
        lam = np.sort(rng.uniform(0.0, 1.0, size=m))[::-1]
    lam = np.asarray(lam, dtype=np.float64)
    Q = haar_orthogonal(rng, m)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return A, Q, lam


def batch_shapes(n_cubes: int = 64, seed: int = 4000):
    """Shapes of the batched workload: (side, bands, r) per cube.

    Square spatial side uniform in {64..512}, bands uniform in {64..256},
    endmembers uniform in {4..12}; cube i draws from default_rng(seed + i).
    """
    out = []
    for i in range(n_cubes):
        rng = np.random.default_rng(seed + i)
        side = int(rng.integers(64, 513))
        bands = int(rng.integers(64, 257))
        r = int(rng.integers(4, 13))
        out.append((side, bands, r))
    return out


def make_config(name: str, seed=None, n_pixels=None, stress: bool = False):
    """Build one workload by name ("c1", "c2", "c3", "c5").

    ``n_pixels`` truncates the pixel count (a leading sample of the same
    generator stream is *not* guaranteed; the cube is regenerated at that
    size). Returns a dict with Y (float32 [N][M], or uint16 for c3 under key
    "Y_u16" plus its float32 conversion under "Y"), k, and shape info.
    """
    cfg = CONFIGS[name]
    if cfg["kind"] == "batch":
        raise ValueError("use make_batch for the batched workload")
    seed = cfg["seed"] if seed is None else seed
    rng = np.random.default_rng(seed)
    n = cfg["h"] * cfg["w"] if n_pixels is None else int(n_pixels)
    m = cfg["bands"]
    out = dict(name=name, k=cfg["k"], n_pixels=n, bands=m, seed=seed)
    if cfg["kind"] == "mixture":
        out["Y"] = mixture_cube(rng, n, m, cfg["r"], cfg["alpha"], cfg["sigma"])
    elif cfg["kind"] == "radiance_u16":
        u = radiance_cube_u16(rng, n, m, cfg["r"], cfg["alpha"])
        out["Y_u16"] = u
        out["Y"] = u.astype(np.float32)
    elif cfg["kind"] == "planted":
        X, Q, lam, mu = planted_cube(rng, n, m, stress=stress)
        out["Y64"] = X
        out["Y"] = X.astype(np.float32)
        out["Q"], out["lam"], out["mu"] = Q, lam, mu
    return out


def make_batch(n_cubes: int = 64, seed: int = 4000, max_side=None):
    """The batched workload: list of float32 cubes with uneven (N, M).

    ``max_side`` caps the spatial side (for quick tests); the shape draws are
    unchanged, only the pixel count is clipped.
    """
    cubes = []
    for i, (side, bands, r) in enumerate(batch_shapes(n_cubes, seed)):
        if max_side is not None:
            side = min(side, max_side)
        rng = np.random.default_rng(seed + 10_000 + i)
        Y = mixture_cube(rng, side * side, bands, r, 1.0, 0.01)
        cubes.append(Y)
    return cubes
