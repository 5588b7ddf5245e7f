"""Properties of the seeded input generators."""

import numpy as np

import synth


def test_seed_reproduces_bitwise():
    a = synth.make_config("c1")["Y"]
    b = synth.make_config("c1")["Y"]
    assert a.dtype == np.float32 and a.shape == (4096, 32)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    c = synth.make_config("c1", seed=7)["Y"]
    assert not np.array_equal(a, c)


def test_endmembers_scaled_to_unit_interval():
    E = synth.endmember_spectra(np.random.default_rng(0), 6, 50)
    assert E.shape == (6, 50)
    assert np.allclose(E.min(axis=1), 0.0) and np.allclose(E.max(axis=1), 1.0)


def test_radiance_cube_is_uint16_in_range():
    u = synth.radiance_cube_u16(np.random.default_rng(1), 2000, 24, 4, 1.0)
    assert u.dtype == np.uint16
    assert u.min() >= 300 and u.max() <= 65535


def test_planted_cube_has_planted_covariance():
    rng = np.random.default_rng(2)
    X, Q, lam, mu = synth.planted_cube(rng, 1000, 10)
    Xc = X - mu
    assert np.max(np.abs(Xc.sum(axis=0))) < 1e-9
    S = Xc.T @ Xc / 999.0
    assert np.max(np.abs(S - (Q * lam) @ Q.T)) < 1e-12
    stress = synth.planted_spectrum(128, stress=True)
    assert np.allclose(-np.diff(stress[:8]), 1e-3)


def test_batch_shapes_in_range():
    shapes = synth.batch_shapes(64)
    assert len(shapes) == 64
    for side, bands, r in shapes:
        assert 64 <= side <= 512 and 64 <= bands <= 256 and 4 <= r <= 12
