"""Pins of the oracle's eigenvector adjoint (``oracle.bse.grad_from_eigvecs``).

The adjoint of a loss that depends on the eigenvectors as well as the
eigenvalues is pinned to things other than itself: central finite
differences through the oracle's Alg. 3 solve (itself pinned in
test_oracle_pins.py), finite differences at 50 digits through mpmath's
eigensolver on tiny problems, the eigenvalue-only adjoint (Thm EValSym part 3,
pinned by closed forms) as the special case G_X = 0, invariances (phase of
each eigenvector, a loss that is constant on the solution set) and an exactly
degenerate spectrum.  The last test plants mistakes in a copy of the adjoint
and checks that the finite-difference pin rejects each.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import bse as ob
from paper_2008_08825_amd import inputs

# Lorentzian spectrum on a small grid (the same form as the full-size loss)
SPEC = dict(n_omega=48, omega_max=12.0, eta=0.4)


def _herm(rng, n):
    return inputs.hermitian_gaussian(rng, n, 1.0)


def _dip(rng, n):
    return rng.standard_normal(2 * n) + 1j * rng.standard_normal(2 * n)


def _loss(A, B, dip):
    lam, X = ob.solve_chol_svd(A, B)
    return ob.oscillator_spectrum_loss(lam, X, dip, **SPEC)


def _grad(A, B, dip, fn=ob.grad_from_eigvecs):
    lam, X = ob.solve_chol_svd(A, B)
    g, GX = ob.oscillator_spectrum_partials(lam, X, dip, **SPEC)
    return fn(lam, X, g, GX)


def _fd_check(A, B, dip, GA, GB, rng, h=1e-4, rtol=1e-7, trials=2):
    """Fourth-order central differences along random Hermitian directions."""
    def d4(f):
        return (8 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h)
    n = A.shape[0]
    worst = 0.0
    for _ in range(trials):
        E = _herm(rng, n)
        F = _herm(rng, n)
        fd = d4(lambda t: _loss(A + t * E, B + t * F, dip))
        an = np.real(np.sum(GA.conj() * E) + np.sum(GB.conj() * F))
        worst = max(worst, abs(fd - an) / max(1.0, abs(an)))
    return worst <= rtol, worst


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (16, 3)])
def test_adjoint_matches_finite_differences(n, seed):
    A, B = inputs.coupled(n, seed=40 + seed, diag_lo=1.0, diag_hi=6.0)
    rng = np.random.default_rng(seed)
    dip = _dip(rng, n)
    GA, GB = _grad(A, B, dip)
    ok, worst = _fd_check(A, B, dip, GA, GB, rng)
    assert ok, worst
    assert np.allclose(GA, GA.conj().T) and np.allclose(GB, GB.conj().T)


def test_adjoint_finite_differences_clustered_spectrum():
    """Near-degenerate pairs (smallest gap ~5e-7 relative): the divided-difference form stays accurate.

    The step stays well above the rounding noise of FP64 eigenvectors inside
    the clusters (about eps ||H|| / gap), which a smaller step would amplify."""
    n = 24
    A, B = inputs.clustered(n, seed=5, clusters=3, width=1e-4, c_norm=1e-4, b_norm=1e-3)
    lam, _ = ob.solve_chol_svd(A, B)
    assert np.min(np.diff(lam)) / lam.max() < 1e-6
    rng = np.random.default_rng(6)
    dip = _dip(rng, n)
    GA, GB = _grad(A, B, dip)
    ok, worst = _fd_check(A, B, dip, GA, GB, np.random.default_rng(7), h=1e-6, rtol=1e-6)
    assert ok, worst


def _mp_eigpairs(H, n):
    """Positive eigenvalues and Sigma-normalised eigenvectors of the mp matrix H1 (2n x 2n)."""
    E, ER = mp.eig(H)
    pos = sorted([k for k in range(2 * n) if mp.re(E[k]) > 0], key=lambda k: mp.re(E[k]))
    lams, vecs = [], []
    for k in pos:
        v = [ER[i, k] for i in range(2 * n)]
        nrm = mp.fsum([abs(v[i]) ** 2 for i in range(n)]) - mp.fsum([abs(v[n + i]) ** 2 for i in range(n)])
        lams.append(mp.re(E[k]))
        vecs.append([x / mp.sqrt(nrm) for x in v])
    return lams, vecs


def _mp_loss(H, n, dip):
    lams, vecs = _mp_eigpairs(H, n)
    om = [(j + mp.mpf(1) / 2) * mp.mpf(SPEC["omega_max"]) / SPEC["n_omega"] for j in range(SPEC["n_omega"])]
    eta = mp.mpf(SPEC["eta"])
    d = [mp.mpc(z.real, z.imag) for z in dip]
    total = mp.mpf(0)
    for lam, v in zip(lams, vecs):
        f = abs(mp.fsum([mp.conj(d[i]) * v[i] for i in range(2 * n)])) ** 2
        total += f * mp.fsum([(eta / mp.pi) / ((w - lam) ** 2 + eta ** 2) for w in om])
    return total


def _mp_h1(A, B, E, F, s, n):
    """H1 of (A + s E, B + s F) at the working precision."""
    def c(z):
        return mp.mpc(complex(z).real, complex(z).imag)
    H = mp.matrix(2 * n, 2 * n)
    for i in range(n):
        for j in range(n):
            a = c(A[i, j]) + s * c(E[i, j])
            b = c(B[i, j]) + s * c(F[i, j])
            H[i, j], H[i, n + j], H[n + i, j], H[n + i, n + j] = a, b, -b, -a
    return H


@pytest.mark.parametrize("n,seed", [(1, 7), (2, 8), (3, 9)])
def test_adjoint_matches_50_digit_finite_differences(n, seed):
    """Brute force on tiny problems: the derivative from mpmath eigenpairs at 50 digits."""
    A, B = inputs.coupled(n, seed=seed, diag_lo=1.0, diag_hi=4.0)
    A = ob.hermitian_from_lower(A)
    B = ob.hermitian_from_lower(B)
    rng = np.random.default_rng(seed)
    dip = _dip(rng, n)
    GA, GB = _grad(A, B, dip)
    E = _herm(rng, n)
    F = _herm(rng, n)
    with mp.workdps(50):
        t = mp.mpf("1e-20")
        fd = (_mp_loss(_mp_h1(A, B, E, F, t, n), n, dip) - _mp_loss(_mp_h1(A, B, E, F, -t, n), n, dip)) / (2 * t)
    an = np.real(np.sum(GA.conj() * E) + np.sum(GB.conj() * F))
    assert abs(float(fd) - an) <= 1e-11 * max(1.0, abs(an))


def test_adjoint_reduces_to_eigenvalue_adjoint():
    """G_X = 0: the eigenvalue-only adjoint of Thm EValSym part 3."""
    A, B = inputs.coupled(11, seed=12)
    lam, X = ob.solve_chol_svd(A, B)
    w = np.random.default_rng(1).standard_normal(11)
    GA, GB = ob.grad_from_eigvecs(lam, X, w, np.zeros_like(X))
    RA, RB = ob.grad_from_eigenpairs(X, w)
    assert np.allclose(GA, RA, atol=1e-13) and np.allclose(GB, RB, atol=1e-13)


def test_adjoint_invariances():
    n = 9
    A, B = inputs.coupled(n, seed=13)
    lam, X = ob.solve_chol_svd(A, B)
    rng = np.random.default_rng(2)
    dip = _dip(rng, n)
    g, GX = ob.oscillator_spectrum_partials(lam, X, dip, **SPEC)
    GA, GB = ob.grad_from_eigvecs(lam, X, g, GX)
    # the phase of each eigenvector is arbitrary: same gradient
    Xp = X * np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    gp, GXp = ob.oscillator_spectrum_partials(lam, Xp, dip, **SPEC)
    GAp, GBp = ob.grad_from_eigvecs(lam, Xp, gp, GXp)
    assert np.allclose(GA, GAp, atol=1e-12) and np.allclose(GB, GBp, atol=1e-12)
    # L = sum_k x_k^H Sigma x_k is n on every solution: zero gradient
    S = np.concatenate([np.ones(n), -np.ones(n)])
    GA0, GB0 = ob.grad_from_eigvecs(lam, X, np.zeros(n), 2 * S[:, None] * X)
    assert np.max(np.abs(GA0)) < 1e-12 and np.max(np.abs(GB0)) < 1e-12


def test_adjoint_exactly_degenerate_cluster():
    """Equal eigenvalues and a loss that sees the cluster through its subspace only."""
    rng = np.random.default_rng(3)
    Q = inputs.haar_unitary(rng, 6)
    a = np.array([2.0, 2.0, 2.0, 3.0, 4.0, 5.0])
    b = np.array([0.5, 0.5, 0.5, 0.7, -0.4, 1.0])
    A = Q.conj().T @ (a[:, None] * Q)
    B = Q.conj().T @ (b[:, None] * Q)
    A = (A + A.conj().T) / 2
    B = (B + B.conj().T) / 2
    lam, X = ob.solve_chol_svd(A, B)
    assert abs(lam[2] - lam[0]) < 1e-14 * lam[-1]
    dip = _dip(rng, 6)
    c = dip.conj() @ X
    GX = 2.0 * np.outer(dip, c)          # L = sum_k |dip^H x_k|^2
    GA, GB = ob.grad_from_eigvecs(lam, X, np.zeros(6), GX)
    assert np.all(np.isfinite(GA)) and np.all(np.isfinite(GB))

    def loss(Ap, Bp):
        _, Xp = ob.solve_chol_svd(Ap, Bp)
        return float(np.sum(np.abs(dip.conj() @ Xp) ** 2))

    h = 1e-5
    for _ in range(2):
        E = _herm(rng, 6)
        F = _herm(rng, 6)
        fd = (loss(A + h * E, B + h * F) - loss(A - h * E, B - h * F)) / (2 * h)
        an = np.real(np.sum(GA.conj() * E) + np.sum(GB.conj() * F))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def _mutant_adjoint(kind):
    """A copy of the oracle's adjoint with one planted mistake."""
    def fn(lam, X, g_lam, G_X):
        n = X.shape[1]
        a, b = X[:n], X[n:]
        Z = np.hstack([X, np.vstack([b, a])])
        l = np.concatenate([lam, -lam])
        s = np.concatenate([np.ones(n), -np.ones(n)])
        Y = Z.conj().T @ G_X
        D = np.zeros((2 * n, n), dtype=complex)
        for k in range(n):
            for i in range(2 * n):
                if i == k:
                    D[i, k] = g_lam[k]
                elif i < n:
                    if kind == "no_conj":        # Y_ik for conj(Y_ik)
                        D[i, k] = (Y[i, k] - Y[k, i]) / (2.0 * (lam[k] - lam[i]))
                    elif kind == "no_half":      # the two combined terms counted twice
                        D[i, k] = (np.conj(Y[i, k]) - Y[k, i]) / (lam[k] - lam[i])
                    else:
                        D[i, k] = (np.conj(Y[i, k]) - Y[k, i]) / (2.0 * (lam[k] - lam[i]))
                elif kind == "no_negative_half":
                    D[i, k] = 0.0
                elif kind == "signature_sign":   # s_i = +1 on the negative half
                    D[i, k] = np.conj(Y[i, k]) / (l[k] - l[i])
                else:
                    D[i, k] = s[i] * np.conj(Y[i, k]) / (l[k] - l[i])
        M = X @ (D.conj().T if kind == "conj_transpose_d" else D.T) @ Z.conj().T
        NA = M[:n, :n] + M[n:, n:]
        NB = M[:n, n:] + M[n:, :n]
        if kind == "swap_ab":                    # blocks of tr(dHcal M) read the wrong way
            NA, NB = NB, NA
        return 0.5 * (NA + NA.conj().T), 0.5 * (NB + NB.conj().T)
    return fn


@pytest.mark.parametrize("kind", ["no_conj", "no_half", "no_negative_half", "signature_sign",
                                  "conj_transpose_d", "swap_ab"])
def test_adjoint_pin_catches_planted_mistakes(kind):
    n = 7
    A, B = inputs.coupled(n, seed=42, diag_lo=1.0, diag_hi=6.0)
    rng = np.random.default_rng(2)
    dip = _dip(rng, n)
    GA, GB = _grad(A, B, dip, fn=_mutant_adjoint("none"))
    assert _fd_check(A, B, dip, GA, GB, np.random.default_rng(9))[0]
    GA, GB = _grad(A, B, dip, fn=_mutant_adjoint(kind))
    assert not _fd_check(A, B, dip, GA, GB, np.random.default_rng(9))[0]
