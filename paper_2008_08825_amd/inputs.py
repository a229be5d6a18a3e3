"""Seeded synthetic inputs for the BSE form-I eigenproblem.

This module draws random matrices and nothing else: it holds none of the
solver's arithmetic, and both the GPU path and the FP64 CPU checker consume
what it returns.  Every generator returns full Hermitian complex128 matrices
``A`` and ``B`` (numpy, row-major) with ``A + B`` and ``A - B`` positive
definite, so that ``H1 = [[A, B], [-B, -A]]`` is a BSE matrix of form I
(Sec. 1, Eq. Hform1) with a positive definite Hamiltonian ``[[A, B], [B, A]]``
(Lemma Qtransform, part 2).

Workload recipes
----------------
``coupled(n, seed, diag_lo, diag_hi, c_norm, b_norm)``
    ``A = diag(D) + C`` with ``D ~ U[diag_lo, diag_hi]`` and ``C`` a random
    Hermitian Gaussian matrix scaled to spectral norm ``c_norm``; ``B`` a random
    Hermitian Gaussian matrix scaled to ``b_norm``.  One ``default_rng(seed)``
    stream, drawn in the order D, C, B.  ``lambda_min(A +- B) >= diag_lo -
    c_norm - b_norm``.
``clustered(n, seed, ...)``
    As ``coupled`` but ``D`` holds 50 clusters of width 1e-3: 50 centres
    ``c_k ~ U[diag_lo, diag_hi]``, then ``k_i ~ U{0..49}``, then
    ``D_i = c_{k_i} + U[-5e-4, 5e-4]``.
``condition_family(n, kappa, seed)``
    The accuracy experiment of Sec. 4 (Table 2): ``A = Q^H diag(d) Q``,
    ``B = A / 2``, ``d`` equally spaced in ``[1, kappa/3]``, ``Q`` Haar unitary.
    The positive eigenvalues are ``(sqrt(3)/2) d`` exactly and ``cond(H1) = kappa``.
``batch_sizes(count, seed)``
    ``count`` problem sizes drawn uniformly from ``{64, ..., 1024}``.

"Random Hermitian Gaussian scaled to spectral norm s": ``X`` with iid N(0,1)
real and imaginary parts, ``G = (X + X^H) / 2``, ``G * s / ||G||_2``.  The
spectral norm is the largest eigenvalue magnitude, from a dense FP64
``eigvalsh`` for ``n <= 2048`` and from Lanczos (ARPACK, all-ones start
vector, residual tolerance 1e-6, so the Ritz value is accurate to about
1e-12 relative) above that, where the dense route takes minutes on a host.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "hermitian_gaussian",
    "coupled",
    "clustered",
    "condition_family",
    "batch_sizes",
    "workload",
    "WORKLOADS",
    "garbage_upper",
]


def _spectral_norm_hermitian(G: np.ndarray) -> float:
    n = G.shape[0]
    if n <= 2048:
        return float(np.max(np.abs(np.linalg.eigvalsh(G))))
    from scipy.sparse.linalg import eigsh

    v0 = np.ones(n, dtype=G.dtype)
    w = eigsh(G, k=1, which="LM", v0=v0, tol=1e-6, return_eigenvectors=False)
    return float(np.abs(w[0]))


def hermitian_gaussian(rng: np.random.Generator, n: int, norm: float,
                       real: bool = False) -> np.ndarray:
    """Random Hermitian matrix with iid Gaussian entries scaled to ``||G||_2 = norm``."""
    if real:
        X = rng.standard_normal((n, n))
        G = (X + X.T) / 2
    else:
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        G = (X + X.conj().T) / 2
    if norm == 0.0 or n == 0:
        return np.zeros((n, n), dtype=G.dtype)
    s = _spectral_norm_hermitian(G)
    return G * (norm / s)


def coupled(n: int, seed: int = 0, diag_lo: float = 1.0, diag_hi: float = 10.0,
            c_norm: float = 0.3, b_norm: float = 0.3, real: bool = False):
    rng = np.random.default_rng(seed)
    D = rng.uniform(diag_lo, diag_hi, size=n)
    C = hermitian_gaussian(rng, n, c_norm, real)
    B = hermitian_gaussian(rng, n, b_norm, real)
    A = C.copy()
    A[np.diag_indices(n)] += D
    return _as_complex(A, real), _as_complex(B, real)


def coupled_form2(n: int, seed: int = 0, diag_lo: float = 1.0, diag_hi: float = 10.0,
                  c_norm: float = 0.3, b_norm: float = 0.3):
    """Form-II input (Eq. Hform2): A Hermitian as in ``coupled``, B complex symmetric
    (B = B^T) of spectral norm about ``b_norm`` (Gaussian, symmetrised), so that the
    Hamiltonian [A B; conj(B) conj(A)] is positive definite when b_norm < diag_lo - c_norm."""
    rng = np.random.default_rng(seed)
    D = rng.uniform(diag_lo, diag_hi, size=n)
    C = hermitian_gaussian(rng, n, c_norm, False)
    A = C.astype(np.complex128)
    A[np.diag_indices(n)] += D
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    S = G + G.T
    nrm = np.linalg.norm(S, 2) if n > 0 else 1.0
    B = S * (b_norm / nrm) if nrm > 0 else S
    return A, B


def clustered(n: int, seed: int = 0, diag_lo: float = 1.0, diag_hi: float = 10.0,
              c_norm: float = 0.3, b_norm: float = 0.3, clusters: int = 50,
              width: float = 1e-3):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(diag_lo, diag_hi, size=clusters)
    k = rng.integers(0, clusters, size=n)
    D = centres[k] + rng.uniform(-width / 2, width / 2, size=n)
    C = hermitian_gaussian(rng, n, c_norm)
    B = hermitian_gaussian(rng, n, b_norm)
    A = C.copy()
    A[np.diag_indices(n)] += D
    return A, B


def haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    Z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    Qm, R = np.linalg.qr(Z)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Qm * ph[None, :]


def condition_family(n: int, kappa: float, seed: int = 0):
    """Sec. 4 accuracy experiment: exact eigenvalues ``sqrt(3)/2 * d``."""
    rng = np.random.default_rng(seed)
    Q = haar_unitary(rng, n)
    d = np.linspace(1.0, kappa / 3.0, n)
    A = Q.conj().T @ (d[:, None] * Q)
    A = (A + A.conj().T) / 2
    B = A / 2
    return A, B, d


def batch_sizes(count: int = 256, seed: int = 0, lo: int = 64, hi: int = 1024):
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(lo, hi + 1, size=count)]


def garbage_upper(M: np.ndarray, seed: int = 12345) -> np.ndarray:
    """Copy of ``M`` whose strict upper triangle and diagonal imaginary parts are noise.

    The solver reads only the lower triangle and the real part of the diagonal,
    so its output must not change.
    """
    rng = np.random.default_rng(seed)
    n = M.shape[0]
    out = M.copy()
    iu = np.triu_indices(n, 1)
    out[iu] = rng.standard_normal(len(iu[0])) * 7 + 1j * rng.standard_normal(len(iu[0])) * 7
    out[np.diag_indices(n)] = out.diagonal().real + 1j * rng.standard_normal(n)
    return out


def _as_complex(M, real):
    return M.astype(np.complex128)


# Named workloads: sizes, value distributions and seeds of the five configurations.
WORKLOADS = {
    "n256": dict(kind="coupled", n=256, diag_lo=2.0, diag_hi=6.0, c_norm=0.5, b_norm=0.5, seed=0),
    "n2048": dict(kind="coupled", n=2048, diag_lo=1.0, diag_hi=10.0, c_norm=0.3, b_norm=0.3, seed=0),
    "n8192_clustered": dict(kind="clustered", n=8192, diag_lo=1.0, diag_hi=10.0, c_norm=0.3,
                            b_norm=0.3, seed=0),
    "n4096": dict(kind="coupled", n=4096, diag_lo=1.0, diag_hi=10.0, c_norm=0.3, b_norm=0.3, seed=0),
}


def workload(name: str, n: int | None = None, seed: int | None = None):
    """Return ``(A, B)`` for a named workload; ``n``/``seed`` override its size/seed."""
    spec = dict(WORKLOADS[name])
    kind = spec.pop("kind")
    if n is not None:
        spec["n"] = n
    if seed is not None:
        spec["seed"] = seed
    if kind == "coupled":
        return coupled(**spec)
    if kind == "clustered":
        return clustered(**spec)
    raise KeyError(name)


def batch_problem(i: int, n: int):
    """Problem ``i`` of the batched workload: the n=2048 recipe at size ``n``, seed 1000+i."""
    return coupled(n, seed=1000 + i, diag_lo=1.0, diag_hi=10.0, c_norm=0.3, b_norm=0.3)
