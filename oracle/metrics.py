"""Error measures used to compare a computed eigen-solution with the oracle (test infrastructure).

All in FP64 numpy.  ``X`` columns are eigenvectors of ``H1`` for the positive
eigenvalues, normalised to ``X^H Sigma X = I`` (Thm ProdEig, Eq. SigmaOrthEVecs).

* relative eigenvalue error ``max_k |lam_k - lam_k^o| / lam_k^o``;
* Sigma-orthogonality ``||X^H Sigma X - I||_F`` (the measure of Fig. 2);
* normalised residual ``||H1 X - X diag(lam)||_F / (||H1||_F ||X||_F)``;
* eigenvector distance: a simple eigenvector is unique up to a phase, so each
  computed vector is phase-aligned with the oracle's before the relative
  difference is taken; inside a cluster (relative gap below ``cluster_rtol``)
  only the invariant subspace is defined, and the distance is that of the
  Sigma-orthogonal projectors ``P = X_c X_c^H Sigma``.
"""
from __future__ import annotations

import numpy as np

from .bse import bse_matrix


def rel_eig_err(lam: np.ndarray, lam_ref: np.ndarray) -> float:
    lam = np.asarray(lam, dtype=np.float64)
    lam_ref = np.asarray(lam_ref, dtype=np.float64)
    if lam.size == 0:
        return 0.0
    return float(np.max(np.abs(lam - lam_ref) / np.abs(lam_ref)))


def sigma_orth_err(X: np.ndarray) -> float:
    n2, k = X.shape
    n = n2 // 2
    G = X[:n].conj().T @ X[:n] - X[n:].conj().T @ X[n:]
    return float(np.linalg.norm(G - np.eye(k)))


def residual(A: np.ndarray, B: np.ndarray, lam: np.ndarray, X: np.ndarray) -> float:
    H = bse_matrix(A, B)
    R = H @ X - X * lam[None, :]
    den = np.linalg.norm(H) * np.linalg.norm(X)
    return float(np.linalg.norm(R) / den) if den > 0 else 0.0


def clusters(lam: np.ndarray, cluster_rtol: float):
    """Group ascending eigenvalues whose neighbours are within ``cluster_rtol`` relative."""
    groups = []
    cur = [0]
    for k in range(1, len(lam)):
        if abs(lam[k] - lam[k - 1]) <= cluster_rtol * max(abs(lam[k]), abs(lam[k - 1])):
            cur.append(k)
        else:
            groups.append(cur)
            cur = [k]
    if len(lam):
        groups.append(cur)
    return groups


def eigvec_errors(lam_ref: np.ndarray, X_ref: np.ndarray, X: np.ndarray,
                  cluster_rtol: float = 1e-6):
    """Per-eigenvalue eigenvector distance and the relative gap to the nearest other eigenvalue.

    Returns ``(err, relgap)``; for members of a cluster ``err`` is the
    projector distance of the whole cluster (divided by sqrt(cluster size))
    and ``relgap`` the gap of the cluster to its neighbours.
    """
    n = X_ref.shape[0] // 2
    sig = np.concatenate([np.ones(n), -np.ones(n)])
    k = len(lam_ref)
    err = np.zeros(k)
    gap = np.full(k, np.inf)
    groups = clusters(lam_ref, cluster_rtol)
    for gi, g in enumerate(groups):
        lo = lam_ref[g[0]]
        hi = lam_ref[g[-1]]
        gl = np.inf
        if gi > 0:
            gl = min(gl, (lo - lam_ref[groups[gi - 1][-1]]) / lo)
        if gi + 1 < len(groups):
            gl = min(gl, (lam_ref[groups[gi + 1][0]] - hi) / hi)
        if len(g) == 1:
            j = g[0]
            xr = X_ref[:, j]
            xc = X[:, j]
            ip = np.vdot(xr, xc)
            ph = ip / abs(ip) if abs(ip) > 0 else 1.0
            e = np.linalg.norm(xc * np.conj(ph) - xr) / np.linalg.norm(xr)
        else:
            Xr = X_ref[:, g]
            Xc = X[:, g]
            Pr = Xr @ (Xr.conj().T * sig[None, :])
            Pc = Xc @ (Xc.conj().T * sig[None, :])
            e = np.linalg.norm(Pr - Pc) / (np.linalg.norm(Pr) + 1e-300)
        err[g] = e
        gap[g] = gl
    return err, gap
