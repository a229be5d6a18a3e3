"""FP64 CPU oracle for the BSE form-I eigenproblem (test infrastructure only).

This package is the slow, plain checker that the GPU solver is measured
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never does.  It shares no code with the
HIP library: every step below is numpy / scipy / mpmath in float64 (or
arbitrary precision), written from the paper.

Problem (Sec. 1, Eq. Hform1; Alg. 3 Require/Ensure): for Hermitian ``A``,
``B`` with ``A + B`` and ``A - B`` positive definite, find the ``n`` positive
eigenvalues ``lambda_1 <= ... <= lambda_n`` of ``H1 = [[A, B], [-B, -A]]`` and
eigenvectors ``X`` (2n x n) with ``H1 X = X diag(lambda)`` and
``X^H Sigma X = I`` (Sec. 4 normalisation; Thm ProdEig Eq. SigmaOrthEVecs).
The negative half is ``-lambda`` with ``[[0, I], [I, 0]] X`` (Lemma
ComputeNegEvecs, part 1).

Input convention shared with the GPU path: only the lower triangle of ``A``
and ``B`` is read and the imaginary part of the diagonal is ignored
(LAPACK ``uplo='L'``).

Routes
------
``solve_chol_svd``  Alg. 3 (CHOL+SVD) with LAPACK ``gesvd``, the primary oracle.
``eigenvalues_chol_svd``  Alg. 3 steps 1-3 only, the eigenvalues (what Table 2
                    times and measures), for sizes where vectors cost too much.
``solve_chol_eig``  Alg. 2 (CHOL) with LAPACK ``heevd``.
``solve_tda``       the Tamm-Dancoff approximation B = 0 (Sec. 4, Table 3).
``solve_sqrt``      Alg. 1 (SQRT), the square-root method the paper compares with.
``solve_pencil``    the Hermitian-definite pencil route (Thm DefiniteRealEvals).
``solve_dense``     nonsymmetric ``eig`` of the full ``H1`` (tiny n only).
``solve_mp``        mpmath eigenvalues of ``H1`` at 50 digits (n <= 6).
``solve_form2``     form II (Eq. Hform2): the Hermitian-definite pencil of its
                    Hamiltonian, the definition of its eigenpairs (no algorithm
                    of the paper is involved).

Paper readings used here: the display of Lemma Qtransform has the two
off-diagonal blocks swapped; direct computation (and the proof of Thm ProdEig)
gives ``Q^-1 H Q = [[0, A+B], [A-B, 0]]``.  The text before Lemma
SVDScalarFactors names ``L1 L2^H`` as the matrix whose SVD is taken; the Lemma
and Alg. 3 use ``L1^H L2``, which is the one whose singular values are the
eigenvalues.  Eigenvalues are returned in ascending order (stable).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = [
    "hermitian_from_lower",
    "bse_matrix",
    "bse_hamiltonian",
    "solve_chol_svd",
    "eigenvalues_chol_svd",
    "solve_chol_eig",
    "solve_tda",
    "solve_sqrt",
    "solve_pencil",
    "solve_dense",
    "solve_mp",
    "negative_half",
    "symmetric_from_lower",
    "bse_matrix_form2",
    "bse_hamiltonian_form2",
    "solve_form2",
    "negative_half_form2",
    "chol_status",
    "grad_from_eigenpairs",
    "spectrum_loss",
    "spectrum_loss_weights",
    "grad_from_eigvecs",
    "oscillator_spectrum_loss",
    "oscillator_spectrum_partials",
]


def hermitian_from_lower(M: np.ndarray) -> np.ndarray:
    """Hermitian matrix defined by the lower triangle of ``M`` (real diagonal)."""
    M = np.asarray(M)
    L = np.tril(M, -1)
    H = L + L.conj().T
    H = H.astype(np.result_type(M.dtype, np.complex128))
    H[np.diag_indices(M.shape[0])] = M.diagonal().real
    return H


def bse_matrix(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """``H1 = [[A, B], [-B, -A]]`` (Eq. Hform1), from the lower triangles of A, B."""
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    return np.block([[A, B], [-B, -A]])


def bse_hamiltonian(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """``Sigma H1 = [[A, B], [B, A]]`` (Eq. BSEHam / Eq. EVform1)."""
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    return np.block([[A, B], [B, A]])


def _assemble(V1: np.ndarray, V2: np.ndarray) -> np.ndarray:
    """Final setup shared by Algs. 1-3: ``V = [(V1 + V2)/2; (V2 - V1)/2]``."""
    return np.vstack([(V1 + V2) / 2, (V2 - V1) / 2])


def solve_chol_svd(A: np.ndarray, B: np.ndarray):
    """Alg. 3 (CHOL+SVD), step by step.

    1. ``L1 L1^H = M1 = A + B``     (Cholesky, LAPACK potrf)
    2. ``L2 L2^H = M2 = A - B``
    3. ``U Lambda V^H = L1^H L2``   (SVD, LAPACK gesvd as in Sec. 3.4)
    4. ``V1 = L1 U Lambda^-1/2``, ``V2 = L2 V Lambda^-1/2``  (Lemma SVDScalarFactors)
    5. ``X = [(V1 + V2)/2; (V2 - V1)/2]``
    Returns ``(lam, X)`` with ``lam`` ascending.
    """
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    M1 = A + B
    M2 = A - B
    L1 = sla.cholesky(M1, lower=True)
    L2 = sla.cholesky(M2, lower=True)
    U, s, Vh = sla.svd(L1.conj().T @ L2, lapack_driver="gesvd")
    V = Vh.conj().T
    V1 = (L1 @ U) * s ** -0.5
    V2 = (L2 @ V) * s ** -0.5
    X = _assemble(V1, V2)
    order = np.argsort(s, kind="stable")
    return s[order], X[:, order]


def eigenvalues_chol_svd(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Alg. 3 steps 1-3 without vectors: the singular values of ``L1^H L2``.

    Sec. 4 measures and times the eigenvalues alone (Table 2); the singular
    values of ``L1^H L2`` are the positive eigenvalues of ``H1`` (Lemma
    SVDScalarFactors / Thm ProdEig: ``M1 M2`` has eigenvalues ``lambda^2``).
    Same LAPACK ``potrf`` and ``gesvd`` as :func:`solve_chol_svd`, with
    ``compute_uv=False``.  Returns the eigenvalues ascending.
    """
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    L1 = sla.cholesky(A + B, lower=True)
    L2 = sla.cholesky(A - B, lower=True)
    s = sla.svd(L1.conj().T @ L2, compute_uv=False, lapack_driver="gesvd")
    return np.sort(s, kind="stable")


def solve_chol_eig(A: np.ndarray, B: np.ndarray):
    """Alg. 2 (CHOL), step by step.

    1. ``L L^H = A - B``
    2. ``M = L^H (A + B) L = V_M D V_M^H``  (Hermitian eigendecomposition)
    3. ``Lambda = D^1/2``
    4. ``V1 = L^-H V_M Lambda^1/2`` (triangular solve), ``V2 = L V_M Lambda^-1/2``
    5. ``X = [(V1 + V2)/2; (V2 - V1)/2]``
    """
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    L = sla.cholesky(A - B, lower=True)
    M = L.conj().T @ (A + B) @ L
    M = (M + M.conj().T) / 2
    d, VM = sla.eigh(M)
    lam = np.sqrt(d)
    V1 = sla.solve_triangular(L.conj().T, VM, lower=False) * np.sqrt(lam)
    V2 = (L @ VM) / np.sqrt(lam)
    X = _assemble(V1, V2)
    order = np.argsort(lam, kind="stable")
    return lam[order], X[:, order]


def solve_sqrt(A: np.ndarray, B: np.ndarray):
    """Alg. 1 (SQRT), step by step (Sec. 3.1, Lemma CrosScalarFactors).

    1. ``S = (A - B)^1/2``, the principal square root, by a Hermitian
       eigendecomposition ``A - B = V_C D_C V_C^H``, ``S = V_C D_C^1/2 V_C^H``
    2. ``M = S (A + B) S = V_M D V_M^H``  (Hermitian eigendecomposition)
    3. ``Lambda = D^1/2``
    4. ``V1 = S^-1 V_M Lambda^1/2``, ``V2 = S V_M Lambda^-1/2``
    5. ``X = [(V1 + V2)/2; (V2 - V1)/2]``
    """
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    dC, VC = sla.eigh(A - B)
    S = (VC * np.sqrt(dC)) @ VC.conj().T
    Sinv = (VC / np.sqrt(dC)) @ VC.conj().T
    M = S @ (A + B) @ S
    M = (M + M.conj().T) / 2
    d, VM = sla.eigh(M)
    lam = np.sqrt(d)
    V1 = (Sinv @ VM) * np.sqrt(lam)
    V2 = (S @ VM) / np.sqrt(lam)
    X = _assemble(V1, V2)
    order = np.argsort(lam, kind="stable")
    return lam[order], X[:, order]


def solve_tda(A: np.ndarray):
    """Tamm-Dancoff approximation (B = 0; Sec. 4 applies it to the LiF matrix, Table 3).

    With ``B = 0``, ``H1 = [[A, 0], [0, -A]]``: the positive eigenpairs are
    those of the Hermitian positive definite ``A`` (``A u = lambda u``) with
    eigenvectors ``[u; 0]``, Sigma-normalised when ``u^H u = 1``.
    """
    A = hermitian_from_lower(A)
    n = A.shape[0]
    lam, U = sla.eigh(A)
    X = np.vstack([U, np.zeros((n, n), dtype=U.dtype)])
    order = np.argsort(lam, kind="stable")
    return lam[order], X[:, order]


def solve_pencil(A: np.ndarray, B: np.ndarray):
    """Hermitian-definite pencil route (proof of Thm DefiniteRealEvals; Sec. 4 "generalized eig").

    ``Sigma z = mu Hcal z`` with ``Hcal = [[A, B], [B, A]]`` positive definite
    and ``z^H Hcal z = 1``; the eigenvalues of ``H1`` are ``1/mu``.  A positive
    eigenpair is rescaled to ``v = z / sqrt(mu)`` so that ``v^H Sigma v = 1``.
    """
    n = A.shape[0]
    Hc = bse_hamiltonian(A, B)
    S = np.diag(np.concatenate([np.ones(n), -np.ones(n)])).astype(np.complex128)
    mu, Z = sla.eigh(S, Hc)
    pos = mu > 0
    lam = 1.0 / mu[pos]
    V = Z[:, pos] / np.sqrt(mu[pos])
    order = np.argsort(lam, kind="stable")
    return lam[order], V[:, order]


def solve_dense(A: np.ndarray, B: np.ndarray):
    """Nonsymmetric eigensolver on the full ``H1`` (Sec. 4 "eig"); tiny n only.

    Keeps the ``n`` eigenvalues with positive real part and scales each
    eigenvector to ``v^H Sigma v = 1``.
    """
    n = A.shape[0]
    H = bse_matrix(A, B)
    w, V = np.linalg.eig(H)
    pos = np.argsort(-w.real, kind="stable")[:n]
    lam = w.real[pos]
    V = V[:, pos]
    sig = np.concatenate([np.ones(n), -np.ones(n)])
    nrm = np.einsum("ik,i,ik->k", V.conj(), sig, V).real
    V = V / np.sqrt(nrm)
    order = np.argsort(lam, kind="stable")
    return lam[order], V[:, order]


def solve_mp(A: np.ndarray, B: np.ndarray, dps: int = 50):
    """Positive eigenvalues of ``H1`` by mpmath's eigensolver at ``dps`` digits (n <= 6)."""
    import mpmath

    H = bse_matrix(A, B)
    n = A.shape[0]
    with mpmath.workdps(dps):
        Hm = mpmath.matrix(2 * n, 2 * n)
        for i in range(2 * n):
            for j in range(2 * n):
                z = complex(H[i, j])
                Hm[i, j] = mpmath.mpc(z.real, z.imag)
        E = mpmath.eig(Hm, left=False, right=False)
        vals = sorted([mpmath.re(e) for e in E], reverse=True)[:n]
        return sorted(vals)


def negative_half(lam: np.ndarray, X: np.ndarray):
    """Lemma ComputeNegEvecs (form I): ``-lambda`` with ``[[0, I], [I, 0]] X``."""
    n = X.shape[0] // 2
    PX = np.vstack([X[n:], X[:n]])
    return -lam, PX


def symmetric_from_lower(M: np.ndarray) -> np.ndarray:
    """Complex symmetric (``M = M^T``, no conjugation) matrix defined by the lower triangle of ``M``."""
    M = np.asarray(M).astype(np.complex128)
    L = np.tril(M, -1)
    return L + L.T + np.diag(M.diagonal())


def bse_matrix_form2(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """``H2 = [[A, B], [-B^H, -A^T]]`` (Eq. Hform2), ``A = A^H``, ``B = B^T``, from lower triangles."""
    A = hermitian_from_lower(A)
    B = symmetric_from_lower(B)
    return np.block([[A, B], [-B.conj().T, -A.T]])


def bse_hamiltonian_form2(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """``Hcal2 = Sigma H2 = [[A, B], [conj(B), conj(A)]]``, Hermitian (positive definite by assumption)."""
    A = hermitian_from_lower(A)
    B = symmetric_from_lower(B)
    return np.block([[A, B], [B.conj(), A.conj()]])


def solve_form2(A: np.ndarray, B: np.ndarray):
    """Positive eigenpairs of a form-II BSE matrix by the Hermitian-definite pencil.

    ``H2 x = lambda x`` with ``H2 = Sigma Hcal2`` is ``Sigma z = mu Hcal2 z`` with
    ``mu = 1 / lambda`` (as the pencil route of form I; the proof of Thm
    DefiniteRealEvals holds for any Hermitian positive definite Hamiltonian).
    LAPACK ``hegv`` returns ``z^H Hcal2 z = 1``; the positive pairs are
    rescaled to ``x = z / sqrt(mu)``, ``x^H Sigma x = 1``.
    """
    n = A.shape[0]
    Hc = bse_hamiltonian_form2(A, B)
    S = np.diag(np.concatenate([np.ones(n), -np.ones(n)])).astype(np.complex128)
    mu, Z = sla.eigh(S, Hc)
    pos = mu > 0
    lam = 1.0 / mu[pos]
    V = Z[:, pos] / np.sqrt(mu[pos])
    order = np.argsort(lam, kind="stable")
    return lam[order], V[:, order]


def negative_half_form2(lam: np.ndarray, X: np.ndarray):
    """Lemma ComputeNegEvecs (form II): ``-lambda`` with ``[[0, I], [I, 0]] conj(X)``."""
    n = X.shape[0] // 2
    PX = np.vstack([X[n:], X[:n]]).conj()
    return -lam, PX


def chol_status(A: np.ndarray, B: np.ndarray) -> int:
    """Status the solver reports for non-HPD input (LAPACK potrf ``info`` convention).

    0 if both ``A + B`` and ``A - B`` are positive definite; ``i`` if the
    leading minor of order ``i`` of ``A + B`` is not; ``n + i`` if ``A + B`` is
    but the leading minor of order ``i`` of ``A - B`` is not (Lemma
    Qtransform, part 2: these are exactly the inputs with indefinite Hamiltonian).
    """
    A = hermitian_from_lower(A)
    B = hermitian_from_lower(B)
    n = A.shape[0]
    _, info1 = sla.lapack.zpotrf(A + B, lower=1)
    if info1 > 0:
        return int(info1)
    _, info2 = sla.lapack.zpotrf(A - B, lower=1)
    if info2 > 0:
        return int(n + info2)
    return 0


def grad_from_eigenpairs(X: np.ndarray, w: np.ndarray):
    """Gradient of ``L = sum_k w_k lambda_k`` with respect to Hermitian ``A`` and ``B``.

    Thm EValSym part 3: for real ``lambda_k`` the left eigenvector is
    ``v_k^H Sigma``, and with ``v_k^H Sigma v_k = 1`` first-order perturbation
    gives ``d lambda_k = v_k^H Sigma dH v_k``.  With ``Sigma dH = [[dA, dB],
    [dB, dA]]`` and ``v_k = [a_k; b_k]`` this is
    ``a^H dA a + b^H dA b + a^H dB b + b^H dB a``, so (convention
    ``dL = Re tr(G^H dA)``)::

        G_A = sum_k w_k (a_k a_k^H + b_k b_k^H)
        G_B = sum_k w_k (a_k b_k^H + b_k a_k^H)
    """
    n = X.shape[0] // 2
    a = X[:n]
    b = X[n:]
    GA = (a * w) @ a.conj().T + (b * w) @ b.conj().T
    GB = (a * w) @ b.conj().T + (b * w) @ a.conj().T
    return GA, GB


def _omegas(n_omega: int, omega_max: float):
    return (np.arange(n_omega) + 0.5) * (omega_max / n_omega)


def spectrum_loss(lam: np.ndarray, k_low: int = 128, n_omega: int = 512,
                  omega_max: float = 12.0, eta: float = 0.05) -> float:
    """Loss of the differentiation workload: lowest-``k_low`` sum plus a Lorentzian spectrum.

    ``L = sum_{k <= k_low} lambda_k + sum_j S(omega_j)`` with
    ``S(omega) = sum_k (eta/pi) / ((omega - lambda_k)^2 + eta^2)`` and
    ``omega_j = (j + 1/2) omega_max / n_omega`` (positive eigenvalues only;
    ``lam`` ascending).
    """
    lam = np.asarray(lam, dtype=np.float64)
    om = _omegas(n_omega, omega_max)
    diff = om[:, None] - lam[None, :]
    S = (eta / np.pi) / (diff ** 2 + eta ** 2)
    return float(lam[:k_low].sum() + S.sum())


def spectrum_loss_weights(lam: np.ndarray, k_low: int = 128, n_omega: int = 512,
                          omega_max: float = 12.0, eta: float = 0.05) -> np.ndarray:
    """``w_k = dL/dlambda_k`` of :func:`spectrum_loss`."""
    lam = np.asarray(lam, dtype=np.float64)
    om = _omegas(n_omega, omega_max)
    diff = om[:, None] - lam[None, :]
    dS = (eta / np.pi) * 2.0 * diff / (diff ** 2 + eta ** 2) ** 2
    w = dS.sum(axis=0)
    w[:k_low] += 1.0
    return w


def grad_from_eigvecs(lam: np.ndarray, X: np.ndarray, g_lam: np.ndarray, G_X: np.ndarray,
                      degen_rtol: float = 1e-13):
    """Gradient of a real loss ``L(lambda, X)`` with respect to Hermitian ``A`` and ``B``.

    ``g_lam = dL/dlambda`` (n) and ``G_X`` (2n x n) with ``dL = Re tr(G_X^H dX)``
    for the columns of ``X`` (positive half, ``X^H Sigma X = I``); returns
    ``(G_A, G_B)`` with ``dL = Re tr(G_A^H dA) + Re tr(G_B^H dB)`` (Hermitian).

    First-order perturbation of the Hermitian pencil ``(Hcal, Sigma)``,
    ``Hcal = Sigma H1 = [[A, B], [B, A]]`` (Eq. BSEHam): with all ``2n``
    eigenvectors ``Z = [X, P X]`` (Lemma ComputeNegEvecs, ``P = [[0, I],
    [I, 0]]``), eigenvalues ``l = [lambda, -lambda]`` and signature
    ``s = [1, ..., 1, -1, ..., -1]``, Thm ProdEig Eq. SigmaOrthEVecs reads
    ``Z^H Sigma Z = diag(s)`` and ``Hcal Z = Sigma Z diag(l)``.  Differentiating,
    with ``K = Z^H dHcal Z`` (Hermitian) and ``dZ = Z C``:
    ``dlambda_k = K_kk`` (Thm EValSym part 3) and, off the diagonal,
    ``C_ik = s_i K_ik / (l_k - l_i)``; the normalisation fixes ``Re C_kk = 0``
    and the phase of each column is held (``C_kk = 0``).  Hence, with
    ``Y = Z^H G_X``,

        dL = Re sum_{i, k <= n} D_ik K_ik,
        D_kk = g_k,
        D_ik = s_i conj(Y_ik) / (l_k - l_i)        (i != k).

    For ``i, k`` both in the positive half the terms ``(i, k)`` and ``(k, i)``
    are combined (``K_ki = conj(K_ik)``) into
    ``D_ik = (conj(Y_ik) - Y_ki) / (2 (lambda_k - lambda_i))`` (the same sum):
    its numerator vanishes for losses invariant under rotations within a
    cluster of equal eigenvalues and is a divided difference for spectral
    functions, so it stays finite as the gap closes.  Pairs with
    ``|lambda_k - lambda_i| <= degen_rtol * max(lambda)`` count as degenerate
    and their term is dropped (exact for losses that see a degenerate cluster
    only through its invariant subspace).  Finally, with
    ``M = X D^T Z^H`` and ``tr(dHcal M) = tr(dA (M11 + M22)) + tr(dB (M12 + M21))``,
    ``G_A`` and ``G_B`` are the Hermitian parts of ``M11 + M22`` and
    ``M12 + M21``.
    """
    lam = np.asarray(lam, dtype=np.float64)
    g_lam = np.asarray(g_lam, dtype=np.float64)
    X = np.asarray(X, dtype=np.complex128)
    G_X = np.asarray(G_X, dtype=np.complex128)
    n = X.shape[1]
    a = X[:n]
    b = X[n:]
    Z = np.hstack([X, np.vstack([b, a])])
    l = np.concatenate([lam, -lam])
    s = np.concatenate([np.ones(n), -np.ones(n)])
    Y = Z.conj().T @ G_X
    tol = degen_rtol * (np.max(np.abs(lam)) if n else 0.0)
    # D[i, k] for i, k in the positive half (rows 0..n-1), entry by entry as above
    Yt = Y[:n]
    gap = lam[None, :] - lam[:, None]                      # gap[i, k] = lambda_k - lambda_i
    off = (np.abs(gap) > tol) & ~np.eye(n, dtype=bool)
    Dt = np.zeros((n, n), dtype=np.complex128)
    Dt[off] = ((np.conj(Yt) - Yt.T) / (2.0 * np.where(off, gap, 1.0)))[off]
    Dt[np.diag_indices(n)] = g_lam
    # the negative half (rows n..2n-1): s_i conj(Y_ik) / (l_k - l_i)
    Db = s[n:, None] * np.conj(Y[n:]) / (l[None, :n] - l[n:, None])
    D = np.vstack([Dt, Db])
    M = X @ D.T @ Z.conj().T
    NA = M[:n, :n] + M[n:, n:]
    NB = M[:n, n:] + M[n:, :n]
    GA = 0.5 * (NA + NA.conj().T)
    GB = 0.5 * (NB + NB.conj().T)
    return GA, GB


def _lorentz(om: np.ndarray, lam: np.ndarray, eta: float):
    """``(phi_k, dphi_k)``: ``sum_j (eta/pi) / ((om_j - lam_k)^2 + eta^2)`` and its lam-derivative."""
    diff = om[:, None] - lam[None, :]
    den = diff ** 2 + eta ** 2
    phi = ((eta / np.pi) / den).sum(axis=0)
    dphi = ((eta / np.pi) * 2.0 * diff / den ** 2).sum(axis=0)
    return phi, dphi


def oscillator_spectrum_loss(lam: np.ndarray, X: np.ndarray, dip: np.ndarray, n_omega: int = 512,
                             omega_max: float = 12.0, eta: float = 0.05) -> float:
    """Absorption-type loss from eigenvalues and eigenvectors (Sec. 1's use of the eigenpairs).

    ``L = sum_j S(omega_j)``, ``S(omega) = sum_k f_k (eta/pi) / ((omega - lambda_k)^2 + eta^2)``
    with oscillator strengths ``f_k = |dip^H X_k|^2`` for a 2n-vector ``dip``
    and ``omega_j = (j + 1/2) omega_max / n_omega``.  ``f_k`` does not depend on
    the phase of ``X_k``.
    """
    lam = np.asarray(lam, dtype=np.float64)
    f = np.abs(np.asarray(dip).conj() @ np.asarray(X)) ** 2
    phi, _ = _lorentz(_omegas(n_omega, omega_max), lam, eta)
    return float((f * phi).sum())


def oscillator_spectrum_partials(lam: np.ndarray, X: np.ndarray, dip: np.ndarray, n_omega: int = 512,
                                 omega_max: float = 12.0, eta: float = 0.05):
    """``(g_lam, G_X)`` of :func:`oscillator_spectrum_loss`.

    ``g_k = f_k phi'(lambda_k)`` and ``G_X[:, k] = 2 dip (dip^H X_k) phi(lambda_k)``,
    so that ``dL = sum_k g_k dlambda_k + Re tr(G_X^H dX)``.
    """
    lam = np.asarray(lam, dtype=np.float64)
    dip = np.asarray(dip, dtype=np.complex128)
    c = dip.conj() @ np.asarray(X)
    phi, dphi = _lorentz(_omegas(n_omega, omega_max), lam, eta)
    g = np.abs(c) ** 2 * dphi
    G_X = 2.0 * np.outer(dip, c * phi)
    return g, G_X
