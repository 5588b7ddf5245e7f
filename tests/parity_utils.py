"""Comparison rules between GPU results and the FP64 oracle.

Readings of the accuracy targets:
  - eigenvalues: normwise, max_i |lam_hat_i - lam_i| / lam_1;
  - eigenvectors: only principal components that are well separated,
    min(lam_{i-1} - lam_i, lam_i - lam_{i+1}) >= g lam_1 with g = 1e-3, are
    compared one by one (angle after aligning signs by the dot product); the
    leading-k subspace is compared through sin(theta_max) when
    lam_k - lam_{k+1} >= g lam_1;
  - projections: per well-separated column i < k, ||Q_hat_i - Q_i|| / ||Q_i||.
"""

from __future__ import annotations

import numpy as np

GAP = 1e-3
# sin(theta_max) of the leading-k subspace, wherever the gap rule applies.
SUBSPACE_TOL = 1e-4


def eig_err(lam_hat, lam):
    lam_hat = np.asarray(lam_hat, dtype=np.float64)
    return float(np.max(np.abs(lam_hat - lam)) / abs(lam[0]))


def well_separated(lam, count, g=GAP):
    lam = np.asarray(lam, dtype=np.float64)
    out = []
    for i in range(count):
        left = lam[i - 1] - lam[i] if i > 0 else np.inf
        right = lam[i] - lam[i + 1] if i + 1 < len(lam) else np.inf
        out.append(min(left, right) >= g * abs(lam[0]))
    return np.array(out)


def vec_angles(V_hat, V, idx):
    V_hat = np.asarray(V_hat, dtype=np.float64)
    out = []
    for i in idx:
        a, b = V_hat[:, i], V[:, i]
        a = a / np.linalg.norm(a)
        c = float(np.dot(a, b))
        r = a - c * b
        out.append(float(np.arctan2(np.linalg.norm(r), abs(c))))
    return np.array(out)


def subspace_sin(Vk_hat, Vk):
    Vk_hat = np.asarray(Vk_hat, dtype=np.float64)
    Qh, _ = np.linalg.qr(Vk_hat)
    R = Qh - Vk @ (Vk.T @ Qh)
    return float(np.linalg.norm(R, 2))


def proj_rel(Q_hat, Q, V_hat, V, idx):
    Q_hat = np.asarray(Q_hat, dtype=np.float64)
    out = []
    for i in idx:
        s = 1.0 if np.dot(V_hat[:, i], V[:, i]) >= 0 else -1.0
        out.append(float(np.linalg.norm(s * Q_hat[:, i] - Q[:, i]) / np.linalg.norm(Q[:, i])))
    return np.array(out)


def sign_rule_holds(V_hat, cols):
    V_hat = np.asarray(V_hat)
    idx = np.argmax(np.abs(V_hat[:, cols]), axis=0)
    return bool(np.all(V_hat[idx, cols] > 0))


def report(lam_hat, V_hat, Q_hat, ref, k, g=GAP):
    """Error summary of one GPU run against an oracle result dict."""
    lam, V, Q = ref["lam"], ref["V"], ref["Q"]
    ws = well_separated(lam, k, g)
    idx = [i for i in range(k) if ws[i]]
    out = dict(eig=eig_err(lam_hat, lam), well_separated=idx)
    out["angle"] = float(vec_angles(V_hat, V, idx).max()) if idx else 0.0
    out["proj"] = float(proj_rel(Q_hat, Q, V_hat, V, idx).max()) if (idx and Q_hat is not None) else 0.0
    if k < len(lam) and (lam[k - 1] - lam[k]) >= g * abs(lam[0]):
        out["subspace"] = subspace_sin(np.asarray(V_hat)[:, :k], V[:, :k])
    return out
