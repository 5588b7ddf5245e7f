"""Independent checks ("pins") of the FP64 oracle.

Each check compares the oracle with something other than itself: exact
rational arithmetic, closed forms of the paper's 2x2 rotation (equations
(2)-(6)), textbook closed forms, LAPACK, planted spectra, and invariants of
the exact decomposition. They are plain functions so that the planted-mistake
tests can run the same checks against deliberately broken oracle variants.
Each raises AssertionError on failure.
"""

from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / scale


# --- band mean and centring ------------------------------------------------
def check_mean_fsum(seed=0, n=5000, m=7, lib=None):
    rng = np.random.default_rng(seed)
    Y = (1000.0 + rng.standard_normal((n, m))).astype(np.float32)
    mu = oracle.band_mean(Y)
    ref = np.array([math.fsum(Y[:, b].astype(np.float64)) / n for b in range(m)])
    assert _rel(mu, ref, 1000.0) <= 1e-13, "band mean differs from the correctly rounded sum"


def check_exact_rational(seed=1, lib=None):
    """Mean and covariance of a tiny cube against exact rational arithmetic."""
    rng = np.random.default_rng(seed)
    n, m = 6, 3
    Y = rng.integers(-50, 50, size=(n, m)).astype(np.float32) / 8.0
    Yq = [[Fraction(float(Y[p, b])) for b in range(m)] for p in range(n)]
    mu_q = [sum(Yq[p][b] for p in range(n)) / n for b in range(m)]
    C_q = [[sum((Yq[p][i] - mu_q[i]) * (Yq[p][j] - mu_q[j]) for p in range(n)) / (n - 1)
            for j in range(m)] for i in range(m)]
    mu = oracle.band_mean(Y)
    C = oracle.covariance(oracle.center(Y, mu))
    assert max(abs(float(mu_q[b]) - mu[b]) for b in range(m)) <= 1e-14
    assert max(abs(float(C_q[i][j]) - C[i, j]) for i in range(m) for j in range(m)) <= 1e-13
    # Entry-by-entry form used for sampled checks of full-size results.
    pairs = [(i, j) for i in range(m) for j in range(m)]
    ent = oracle.covariance_entries(Y, mu, pairs)
    assert max(abs(float(C_q[i][j]) - e) for (i, j), e in zip(pairs, ent)) <= 1e-13, \
        "covariance entries differ from exact rational arithmetic"


# --- covariance ------------------------------------------------------------
def check_cov_numpy(seed=2, lib=None):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((3000, 9)) * rng.uniform(0.5, 3, size=9) + 5.0
    C = oracle.covariance(oracle.center(Y))
    ref = np.cov(Y, rowvar=False, ddof=1)
    assert _rel(C, ref, np.abs(ref).max()) <= 1e-12, "covariance differs from numpy.cov"
    assert np.array_equal(C, C.T), "covariance not exactly symmetric"
    assert np.linalg.eigvalsh(C).min() >= -1e-14 * np.abs(ref).max(), "covariance not PSD"


def check_cov_planted(seed=3, n=4000, m=12, lib=None):
    rng = np.random.default_rng(seed)
    X, Q, lam, mu = synth.planted_cube(rng, n, m)
    C = oracle.covariance(oracle.center(X))
    ref = (Q * lam) @ Q.T
    assert _rel(C, ref, lam.max()) <= 1e-12, "planted covariance not recovered"
    mu_o = oracle.band_mean(X)
    assert _rel(mu_o, mu, 1.0) <= 1e-13, "planted mean not recovered"


# --- the 2x2 rotation of equations (1)-(6) ---------------------------------
def check_rotation_2x2(lib=None):
    cases = [(3.0, 1.0, 1.0), (1.0, 0.3, 4.0), (2.0, -1.5, 2.0), (5.0, 1e-3, -2.0),
             (-1.0, 2.0, 7.0), (1.0, 1e-9, 1.0 + 1e-7)]
    for a, b, c in cases:
        A = np.array([[a, b], [b, c]])
        d, E, info = oracle.jacobi_raw(A, tol=1e-15, lib_path=lib)
        if a == c:
            t = 1.0
        else:
            mm = 2.0 * b / (c - a)                                   # eq (2)
            t = (-1.0 + math.sqrt(1.0 + mm * mm)) / mm               # eq (3)
        cos = 1.0 / math.sqrt(1.0 + t * t)                           # eq (4)
        sin = t * cos                                                # eq (5)
        P = np.array([[cos, sin], [-sin, cos]])                      # eq (6)
        B = P.T @ A @ P                                              # eq (1)/(8)
        assert abs(B[0, 1]) <= 1e-12 * (abs(a) + abs(b) + abs(c)), "eqs (2)-(5) do not diagonalise"
        assert _rel(E, P, 1.0) <= 1e-12, "eigenvector matrix is not P of eq (6)"
        assert _rel(d, np.diag(B), abs(a) + abs(b) + abs(c)) <= 1e-12
        lo = (a + c) / 2 - math.sqrt(((a - c) / 2) ** 2 + b * b)
        hi = (a + c) / 2 + math.sqrt(((a - c) / 2) ** 2 + b * b)
        assert _rel(np.sort(d), [lo, hi], abs(a) + abs(b) + abs(c)) <= 1e-12
        assert info["rotations"] == 1 and info["sweeps"] == 1
    d, E, info = oracle.jacobi_raw(np.diag([1.0, 5.0]), lib_path=lib)
    assert info["rotations"] == 0 and info["sweeps"] == 0 and np.array_equal(E, np.eye(2))


# --- eigenvalues against closed forms, brute force and LAPACK ---------------
def check_golden(lib=None):
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        A = np.array(case["A"])
        lam, V, _ = oracle.jacobi_eigh(A, tol=1e-15, lib_path=lib)
        ref = np.array(case["eigvals"])
        assert _rel(lam, ref, np.abs(ref).max()) <= 1e-14, case["name"]
        assert _rel(A @ V, V * lam, np.abs(ref).max()) <= 1e-13, case["name"]


def _cubic_eigs(A):
    """Eigenvalues of a symmetric 3x3 by the trigonometric solution of its
    characteristic cubic (Smith, CACM 4(4), 1961)."""
    q = np.trace(A) / 3.0
    p1 = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
    p2 = (A[0, 0] - q) ** 2 + (A[1, 1] - q) ** 2 + (A[2, 2] - q) ** 2 + 2 * p1
    p = math.sqrt(p2 / 6.0)
    Bm = (A - q * np.eye(3)) / p
    r = np.linalg.det(Bm) / 2.0
    phi = math.acos(min(1.0, max(-1.0, r))) / 3.0
    e1 = q + 2 * p * math.cos(phi)
    e3 = q + 2 * p * math.cos(phi + 2 * math.pi / 3)
    return np.array([e1, 3 * q - e1 - e3, e3])


def check_3x3_trig(seed=4, lib=None):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        G = rng.standard_normal((3, 3))
        A = G + G.T
        lam, _, _ = oracle.jacobi_eigh(A, tol=1e-15, lib_path=lib)
        assert _rel(lam, _cubic_eigs(A), np.abs(lam).max()) <= 1e-12


def check_lapack(seed=5, lib=None):
    rng = np.random.default_rng(seed)
    for n in (2, 3, 5, 8, 17, 32, 64):
        G = rng.standard_normal((n, n))
        A = G + G.T
        lam, V, info = oracle.jacobi_eigh(A, tol=1e-14, lib_path=lib)
        ref = np.linalg.eigvalsh(A)[::-1]
        nrm = np.linalg.norm(A, 2)
        assert info["converged"]
        assert _rel(lam, ref, nrm) <= 1e-12, f"n={n} eigenvalues differ from LAPACK"
        assert _rel(V.T @ V, np.eye(n), 1.0) <= 1e-12, f"n={n} V not orthogonal"
        assert np.linalg.norm(A @ V - V * lam) / np.linalg.norm(A) <= 1e-12, f"n={n} residual"


def check_planted_spectrum(seed=6, m=24, lib=None):
    rng = np.random.default_rng(seed)
    lam0 = np.linspace(2.0, 0.1, m)
    A, Q, lam0 = synth.random_symmetric(rng, m, lam0)
    lam, V, _ = oracle.jacobi_eigh(A, tol=1e-14, lib_path=lib)
    assert _rel(lam, lam0, 2.0) <= 1e-12, "planted eigenvalues not recovered"
    align = np.abs(np.sum(V * Q, axis=0))
    assert np.max(np.abs(align - 1.0)) <= 1e-10, "planted eigenvectors not recovered"
    assert abs(lam.sum() - np.trace(A)) <= 1e-12 * m, "trace not preserved"
    assert abs(np.sum(lam ** 2) - np.sum(A * A)) <= 1e-12 * np.sum(A * A), "Frobenius norm not preserved"


def check_orderings(seed=7, m=20, lib=None):
    rng = np.random.default_rng(seed)
    lam0 = np.linspace(1.0, 0.05, m)
    A, _, _ = synth.random_symmetric(rng, m, lam0)
    base_l, base_v, _ = oracle.jacobi_eigh(A, tol=1e-14, ordering="row", lib_path=lib)
    for ordering in ("round_robin", "classical", "greedy"):
        l2, v2, info = oracle.jacobi_eigh(A, tol=1e-14, ordering=ordering, lib_path=lib)
        assert info["converged"], ordering
        assert _rel(l2, base_l, 1.0) <= 1e-12, ordering
        assert _rel(v2, base_v, 1.0) <= 1e-9, ordering


def check_diagonal_input(lib=None):
    d = np.array([3.0, -1.0, 7.0, 7.0, 0.5])
    lam, V, info = oracle.jacobi_eigh(np.diag(d), lib_path=lib)
    assert info["sweeps"] == 0 and info["rotations"] == 0
    assert np.array_equal(lam, [7.0, 7.0, 3.0, 0.5, -1.0])
    assert np.array_equal(V, np.eye(5)[:, [2, 3, 0, 4, 1]]), "stable order of equal eigenvalues"


def check_sort_and_sign(seed=8, lib=None):
    rng = np.random.default_rng(seed)
    A, _, _ = synth.random_symmetric(rng, 10)
    lam, V, _ = oracle.jacobi_eigh(A, lib_path=lib)
    assert np.all(np.diff(lam) <= 0), "eigenvalues not descending"
    idx = np.argmax(np.abs(V), axis=0)
    assert np.all(V[idx, np.arange(10)] > 0), "sign rule violated"
    # Exact ties: [[a, b], [b, a]] blocks have eigenvectors (1, -1)/sqrt(2)
    # (eigenvalue a - b) and (1, 1)/sqrt(2) (a + b), whose two entries have
    # equal magnitude bit for bit (the rotation of a 45 degree angle has
    # cos == sin). The sign rule then makes the lower index positive.
    r = 1.0 / math.sqrt(2.0)
    lam, V, _ = oracle.jacobi_eigh(np.array([[2.0, -1.0], [-1.0, 2.0]]), lib_path=lib)
    assert np.array_equal(lam, [3.0, 1.0]) or _rel(lam, [3.0, 1.0], 3.0) <= 1e-15
    assert _rel(V, [[r, r], [-r, r]], 1.0) <= 1e-15, "tie in the sign rule not resolved to the lowest index"
    B = np.zeros((4, 4))
    B[:2, :2] = [[5.0, 2.0], [2.0, 5.0]]      # eigenvalues 7 and 3
    B[2:, 2:] = [[1.0, -0.5], [-0.5, 1.0]]    # eigenvalues 1.5 and 0.5
    lam, V, _ = oracle.jacobi_eigh(B, lib_path=lib)
    ref = np.array([[r, r, 0, 0], [r, -r, 0, 0], [0, 0, r, r], [0, 0, -r, r]])
    assert _rel(lam, [7.0, 3.0, 1.5, 0.5], 7.0) <= 1e-15
    assert _rel(V, ref, 1.0) <= 1e-15, "tie in the sign rule not resolved to the lowest index"


# --- projection and loss -----------------------------------------------------
def check_projection_identity(seed=9, lib=None):
    rng = np.random.default_rng(seed)
    Y = synth.mixture_cube(rng, 3000, 16, 5, 1.0, 0.01)
    k = 4
    r = oracle.pca(Y, k, tol=1e-14, lib_path=lib)
    Q = r["Q"]
    n = Q.shape[0]
    G = Q.T @ Q / (n - 1)
    assert _rel(G, np.diag(r["lam"][:k]), r["lam"][0]) <= 1e-12, "Q^T Q/(N-1) != diag(lam)"
    assert np.max(np.abs(Q.sum(axis=0))) <= 1e-9 * np.abs(Q).max() * n ** 0.5
    # The row-by-row form used for sampled checks of full-size results: the
    # same identity over every row.
    Qr = oracle.project_rows(Y, r["mean"], r["V"], k, np.arange(n))
    Gr = Qr.T @ Qr / (n - 1)
    assert _rel(Gr, np.diag(r["lam"][:k]), r["lam"][0]) <= 1e-12, "row-wise Q^T Q/(N-1) != diag(lam)"
    assert np.max(np.abs(Qr.sum(axis=0))) <= 1e-9 * np.abs(Qr).max() * n ** 0.5
    loss = oracle.reconstruction_loss(Y, k, res=r)
    closed = (n - 1) * (np.trace(r["C"]) - r["lam"][:k].sum())
    assert abs(loss - closed) <= 1e-10 * abs(closed), "reconstruction loss closed form"


def check_reconstruction_gradient(seed=10, lib=None):
    """dL/dY = 2 X (I - V_k V_k^T) for L = ||X - Q V_k^T||^2 = ||X||^2 - ||Q||^2."""
    rng = np.random.default_rng(seed)
    X0, _, _, _ = synth.planted_cube(rng, 200, 8)
    k = 3
    r = oracle.pca(X0, k, tol=1e-15, lib_path=lib)
    X, V, Q = r["X"], r["V"], r["Q"]
    g = oracle.backward(X0, k, dQ=-2.0 * Q, res=r) + 2.0 * X
    closed = 2.0 * X @ (np.eye(8) - V[:, :k] @ V[:, :k].T)
    assert _rel(g, closed, np.abs(closed).max()) <= 1e-10


def check_gradient_fd(seed=11, lib=None):
    """Directional derivatives of L = <W, Q> + <w, lam> + <U, V_k> + <z, mu>
    against central finite differences in float64."""
    rng = np.random.default_rng(seed)
    lam0 = np.array([4.0, 2.5, 1.5, 0.9, 0.5, 0.2])
    n, m, k = 60, 6, 3
    X0, _, _, _ = synth.planted_cube(rng, n, m, lam=lam0)
    W = rng.standard_normal((n, k))
    w = rng.standard_normal(m)
    U = rng.standard_normal((m, k))
    z = rng.standard_normal(m)

    def loss(Y):
        r = oracle.pca(Y, k, tol=1e-15, lib_path=lib)
        return (np.sum(W * r["Q"]) + np.dot(w, r["lam"]) + np.sum(U * r["V"][:, :k])
                + np.dot(z, r["mean"]))

    r = oracle.pca(X0, k, tol=1e-15, lib_path=lib)
    G = oracle.backward(X0, k, dQ=W, dlam=w, dVk=U, dmu=z, res=r)
    h = 1e-6
    for _ in range(6):
        D = rng.standard_normal((n, m))
        fd = (loss(X0 + h * D) - loss(X0 - h * D)) / (2 * h)
        an = np.sum(G * D)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


ALL_CHECKS = [
    check_mean_fsum, check_exact_rational, check_cov_numpy, check_cov_planted,
    check_rotation_2x2, check_golden, check_3x3_trig, check_lapack,
    check_planted_spectrum, check_orderings, check_diagonal_input, check_sort_and_sign,
    check_projection_identity, check_reconstruction_gradient, check_gradient_fd,
]
