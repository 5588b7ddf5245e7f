"""Planted mistakes in the oracle must fail at least one pin.

Each case breaks the oracle on the CPU in one plausible way (a wrong sign, a
dropped term, a transposed operand, a wrong normalisation) and runs the pins
of ``oracle_checks`` against it. A case that no pin catches would mean the
pins do not constrain that part of the oracle.
"""

import numpy as np
import pytest

import oracle
import oracle.pca_oracle as po
import oracle_checks as oc


def _first_failure(lib=None):
    for check in oc.ALL_CHECKS:
        try:
            check(lib=lib)
        except Exception as exc:  # AssertionError or a numerical breakdown
            return f"{check.__name__}: {type(exc).__name__}"
    return None


C_MUTANTS = ["ORACLE_MUTANT_TANGENT_SIGN", "ORACLE_MUTANT_DROP_TERM",
             "ORACLE_MUTANT_TRANSPOSED_V"]


@pytest.mark.parametrize("define", C_MUTANTS)
def test_c_mutant_is_caught(define, tmp_path):
    lib = oracle.build_library(defines=[define], out=str(tmp_path / f"{define}.so"))
    assert _first_failure(lib) is not None, f"{define} passes every pin"


def _cov_over_n(X):
    X = np.asarray(X, dtype=np.float64)
    return (X.T @ X) / X.shape[0]


def _center_plus(Y, mu=None):
    Y = po._f64(Y)
    mu = po.band_mean(Y) if mu is None else mu
    return Y + mu[None, :]


def _mean_over_n1(Y):
    Y = po._f64(Y)
    return Y.sum(axis=0) / (Y.shape[0] - 1)


def _sort_ascending(lam, V):
    order = np.argsort(np.asarray(lam), kind="stable")
    return np.asarray(lam)[order], np.asarray(V)[:, order]


def _sign_negative(V):
    return -po.sign_fix.__wrapped__(V) if hasattr(po.sign_fix, "__wrapped__") else -_ORIG["sign_fix"](V)


def _sign_ties_last(V):
    V = np.array(V, dtype=np.float64, copy=True)
    a = np.abs(V)[::-1]
    idx = V.shape[0] - 1 - np.argmax(a, axis=0)      # last index of the maximum
    sgn = np.where(V[idx, np.arange(V.shape[1])] < 0, -1.0, 1.0)
    return V * sgn[None, :]


def _cov_entries_over_n(Y, mu, pairs):
    Y = np.asarray(Y, dtype=np.float64)
    return np.array([np.dot(Y[:, i] - mu[i], Y[:, j] - mu[j]) / Y.shape[0] for i, j in pairs])


def _project_rows_uncentred(Y, mu, V, k, rows):
    return np.asarray(Y, dtype=np.float64)[np.asarray(rows)] @ np.asarray(V, dtype=np.float64)[:, :k]


def _project_rows(X, V, k):
    return np.asarray(X, dtype=np.float64) @ np.asarray(V, dtype=np.float64)[:k, :].T


def _eigh_adjoint_flipped(lam, V, lbar, Vbar):
    return _ORIG["_eigh_adjoint"](-lam, V, lbar, Vbar)


def _eigh_adjoint_unsym(lam, V, lbar, Vbar):
    m = lam.shape[0]
    diff = lam[None, :] - lam[:, None]
    with np.errstate(divide="ignore"):
        F = np.where(np.eye(m, dtype=bool), 0.0, 1.0 / np.where(diff == 0, np.inf, diff))
    return V @ (np.diag(lbar) + F * (V.T @ Vbar)) @ V.T


def _centre_adjoint_identity(Xbar):
    return Xbar


_ORIG = {name: getattr(po, name) for name in
         ("covariance", "center", "band_mean", "sort_desc", "sign_fix", "project",
          "_eigh_adjoint", "_centre_adjoint", "covariance_entries", "project_rows")}

PY_MUTANTS = {
    "covariance divided by N": ("covariance", _cov_over_n),
    "mean added instead of removed": ("center", _center_plus),
    "mean divided by N-1": ("band_mean", _mean_over_n1),
    "eigenvalues sorted ascending": ("sort_desc", _sort_ascending),
    "sign rule inverted": ("sign_fix", _sign_negative),
    "sign rule ties resolved to the last index": ("sign_fix", _sign_ties_last),
    "covariance entries divided by N": ("covariance_entries", _cov_entries_over_n),
    "row-wise projection without centring": ("project_rows", _project_rows_uncentred),
    "projection on rows of V": ("project", _project_rows),
    "eigengap weights with the wrong sign": ("_eigh_adjoint", _eigh_adjoint_flipped),
    "eigh adjoint not symmetrised": ("_eigh_adjoint", _eigh_adjoint_unsym),
    "centring adjoint dropped": ("_centre_adjoint", _centre_adjoint_identity),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_mutant_is_caught(name, monkeypatch):
    target, repl = PY_MUTANTS[name]
    monkeypatch.setattr(po, target, repl)
    if hasattr(oracle, target):
        monkeypatch.setattr(oracle, target, repl)
    assert _first_failure() is not None, f"mutant '{name}' passes every pin"
