"""FP64 reference implementation of the paper's PCA (Algorithm 1, Section 2).

TEST INFRASTRUCTURE ONLY: see the package docstring. Everything here runs on
the host in float64. Library primitives (numpy sums and matrix products) serve
as single steps; the Jacobi sweeps themselves run in the plain C file
``jacobi.c`` next to this one, compiled with gcc on first use.

Stages, in the paper's order:
  1. band-average removal, X = Y - 1 mu^T                (Algorithm 1, line 2)
  2. covariance C = X^T X, normalised by N-1             (Algorithm 1, line 3;
                                                          Section 4, Code 4.3)
  3. eigenvectors of C by cyclic Jacobi                  (Algorithm 1, line 4;
                                                          equations (2)-(10))
  4. eigenvalues sorted in descending order, eigenvector
     columns permuted to match                           (Section 4, Code 4.4.3)
  5. projection onto the first k eigenvectors            (Algorithm 1, lines 5-6)

Readings where the paper is silent or inconsistent (also listed in the design
notes): the covariance is divided by N-1 (as in Code 4.3); the projection uses
the centred cube X (as the GPU design does after its in-place mean
subtraction) rather than the raw Y of Algorithm 1, line 5; the stop factor is a
relative off-norm; ties in the sort keep index order; each eigenvector's sign
is fixed so that its largest-magnitude entry is positive (lowest index on
ties).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB = os.path.join(_HERE, "libjacobi_oracle.so")

ORDERINGS = {"row": 0, "round_robin": 1, "classical": 2, "greedy": 3}

_lib_cache = {}


def build_library(defines=(), out=None) -> str:
    """Compile ``jacobi.c`` with gcc (no fast-math: operations run in the
    written order). ``defines`` builds a planted-mistake variant for the
    tests that check the pins; ``out`` names its output file."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", _SRC, "-o", out + ".tmp", "-lm"]
    cmd[1:1] = ["-D" + d for d in defines]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load(path=None):
    path = path or _LIB
    if path in _lib_cache:
        return _lib_cache[path]
    if path == _LIB and (not os.path.exists(_LIB)
                         or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build_library()
    lib = ctypes.CDLL(path)
    fn = lib.oracle_jacobi
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                   ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                   ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]
    _lib_cache[path] = lib
    return lib


def _f64(Y) -> np.ndarray:
    """The cube as float64 (exact for float32 and uint16 input)."""
    return np.ascontiguousarray(np.asarray(Y), dtype=np.float64)


# ---------------------------------------------------------------------------
# 1. Band-average removal (Algorithm 1, line 2; Section 4 Code 4.2.1-4.2.2 and
#    Section 5 Code 5.1 compute the per-band average and subtract it)
# ---------------------------------------------------------------------------
def band_mean(Y) -> np.ndarray:
    """mu_b = (1/N) sum_p Y[p, b], accumulated in float64."""
    Y = _f64(Y)
    return Y.sum(axis=0) / Y.shape[0]


def center(Y, mu=None) -> np.ndarray:
    """X = Y - 1 mu^T (float64)."""
    Y = _f64(Y)
    if mu is None:
        mu = band_mean(Y)
    return Y - mu[None, :]


# ---------------------------------------------------------------------------
# 2. Covariance (Algorithm 1, line 3; normalisation by PIXELS-1 of Code 4.3)
# ---------------------------------------------------------------------------
def covariance(X) -> np.ndarray:
    """C = X^T X / (N - 1). Only the upper triangle is taken from the product
    and mirrored, as the manycore design computes half of the symmetric
    matrix; the result is exactly symmetric."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    P = X.T @ X
    U = np.triu(P)
    return (U + np.triu(U, 1).T) / (n - 1.0)


def covariance_entries(Y, mu, pairs) -> np.ndarray:
    """Selected entries C[i, j] = sum_p (y_pi - mu_i)(y_pj - mu_j) / (N - 1),
    each computed on its own (for checks of full-size results)."""
    Y = np.asarray(Y)
    n = Y.shape[0]
    out = np.empty(len(pairs))
    cols = {}
    for idx, (i, j) in enumerate(pairs):
        for b in (i, j):
            if b not in cols:
                cols[b] = Y[:, b].astype(np.float64) - mu[b]
        out[idx] = np.dot(cols[i], cols[j]) / (n - 1.0)
    return out


# ---------------------------------------------------------------------------
# 3. Jacobi eigendecomposition (equations (2)-(10); C implementation)
# ---------------------------------------------------------------------------
def jacobi_raw(C, tol=1e-12, max_sweeps=50, ordering="row", lib_path=None):
    """Run the Jacobi iteration on a copy of C.

    Returns (diag of the final iterate, E, info) with E's column j the
    eigenvector of diagonal entry j (unsorted, unsigned)."""
    A = np.array(C, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("C must be square")
    V = np.empty((n, n), dtype=np.float64)
    sweeps = ctypes.c_int(0)
    rots = ctypes.c_longlong(0)
    off = ctypes.c_double(0.0)
    lib = _load(lib_path)
    conv = lib.oracle_jacobi(A.ctypes.data, V.ctypes.data, n, float(tol), int(max_sweeps),
                             ORDERINGS[ordering], ctypes.byref(sweeps), ctypes.byref(rots),
                             ctypes.byref(off))
    if conv < 0:
        raise ValueError("unknown ordering")
    info = dict(converged=bool(conv), sweeps=sweeps.value, rotations=rots.value,
                off_rel=off.value, final=A)
    return np.diag(A).copy(), V, info


# ---------------------------------------------------------------------------
# 4. Sorting and sign convention (Section 4, Code 4.4.3)
# ---------------------------------------------------------------------------
def sort_desc(lam, V):
    """Eigenvalues in descending order (stable: equal values keep index
    order) and eigenvector columns permuted to match."""
    order = np.argsort(-np.asarray(lam), kind="stable")
    return np.asarray(lam)[order], np.asarray(V)[:, order]


def sign_fix(V) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive
    (the first such entry on ties)."""
    V = np.array(V, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.where(V[idx, np.arange(V.shape[1])] < 0, -1.0, 1.0)
    return V * sgn[None, :]


def jacobi_eigh(C, tol=1e-12, max_sweeps=50, ordering="row", lib_path=None):
    """Eigenpairs of the symmetric C: (lam descending, V sign-fixed, info)."""
    lam, V, info = jacobi_raw(C, tol, max_sweeps, ordering, lib_path)
    lam, V = sort_desc(lam, V)
    return lam, sign_fix(V), info


# ---------------------------------------------------------------------------
# 5. Projection and column removal (Algorithm 1, lines 5-6)
# ---------------------------------------------------------------------------
def project(X, V, k) -> np.ndarray:
    """Q' = X V[:, :k] (the first k principal components of every pixel)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(V, dtype=np.float64)[:, :k]


def project_rows(Y, mu, V, k, rows) -> np.ndarray:
    """Q'[rows] computed row by row from the raw cube (for full-size checks)."""
    Y = np.asarray(Y)
    Xr = Y[np.asarray(rows)].astype(np.float64) - mu[None, :]
    return Xr @ np.asarray(V, dtype=np.float64)[:, :k]


def pca(Y, k, tol=1e-12, max_sweeps=50, ordering="row", lib_path=None):
    """Algorithm 1 end to end. Returns a dict with mean, C, lam, V, Q, info."""
    mu = band_mean(Y)
    X = center(Y, mu)
    C = covariance(X)
    lam, V, info = jacobi_eigh(C, tol, max_sweeps, ordering, lib_path)
    Q = project(X, V, k)
    return dict(mean=mu, X=X, C=C, lam=lam, V=V, Q=Q, info=info, k=k)


# ---------------------------------------------------------------------------
# Adjoint of the whole pipeline (reverse-mode derivative)
# ---------------------------------------------------------------------------
def backward(Y, k, dQ=None, dlam=None, dVk=None, dmu=None, res=None):
    """Gradient of a scalar loss with respect to Y, given the loss's gradients
    with respect to the outputs Q (N x k), lam (M), V[:, :k] (M x k) and mu (M).

    Steps in reverse order of the forward pass:
      projection  Q = X V_k:        Xbar = Qbar V_k^T,  Vbar_k += X^T Qbar
      eigenpairs  C = V diag(lam) V^T (distinct eigenvalues):
                  Cbar = V (diag(lambar) + F o (V^T Vbar)) V^T,
                  F_ij = 1/(lam_j - lam_i) for i != j, F_ii = 0,
                  then the symmetric part of Cbar
      covariance  C = X^T X/(N-1):  Xbar += X (Cbar + Cbar^T)/(N-1)
      centring    X = Y - 1 mu^T, mu = 1^T Y / N:
                  Ybar = Xbar - (1/N) 1 1^T Xbar + (1/N) 1 mubar^T
    """
    if res is None:
        res = pca(Y, k)
    X, lam, V = res["X"], res["lam"], res["V"]
    n, m = X.shape
    Xbar = np.zeros_like(X)
    Vbar = np.zeros((m, m))
    if dQ is not None:
        dQ = np.asarray(dQ, dtype=np.float64)
        Xbar += dQ @ V[:, :k].T
        Vbar[:, :k] += X.T @ dQ
    if dVk is not None:
        Vbar[:, :k] += np.asarray(dVk, dtype=np.float64)
    lbar = np.zeros(m) if dlam is None else np.asarray(dlam, dtype=np.float64)
    Cbar = _eigh_adjoint(lam, V, lbar, Vbar)
    Xbar += X @ (2.0 * Cbar) / (n - 1.0)
    Ybar = _centre_adjoint(Xbar)
    if dmu is not None:
        Ybar += np.asarray(dmu, dtype=np.float64)[None, :] / n
    return Ybar


def _eigh_adjoint(lam, V, lbar, Vbar):
    """Cbar = sym(V (diag(lambar) + F o (V^T Vbar)) V^T), F_ij = 1/(lam_j - lam_i)."""
    m = lam.shape[0]
    diff = lam[None, :] - lam[:, None]            # diff[i, j] = lam_j - lam_i
    with np.errstate(divide="ignore"):
        F = np.where(np.eye(m, dtype=bool), 0.0, 1.0 / np.where(diff == 0, np.inf, diff))
    inner = np.diag(lbar) + F * (V.T @ Vbar)
    Cbar = V @ inner @ V.T
    return 0.5 * (Cbar + Cbar.T)


def _centre_adjoint(Xbar):
    """Ybar = (I - 1 1^T / N) Xbar for X = Y - 1 mu^T with mu = 1^T Y / N."""
    return Xbar - Xbar.sum(axis=0)[None, :] / Xbar.shape[0]


def reconstruction_loss(Y, k, res=None) -> float:
    """Squared reconstruction error from the first k components,
    || X - Q' V_k^T ||_F^2."""
    if res is None:
        res = pca(Y, k)
    R = res["X"] - res["Q"] @ res["V"][:, :k].T
    return float(np.sum(R * R))


if __name__ == "__main__":  # pragma: no cover - manual build helper
    print(build_library())
    sys.exit(0)
