"""Pins of the oracle's form-II solver (Eq. Hform2, Thm Form2) against closed forms and brute force.

The paper gives the structure of form II (``H2 = [A B; -B^H -A^T]``, ``A``
Hermitian, ``B`` complex symmetric) but no algorithm; the oracle takes the
Hermitian-definite pencil of its Hamiltonian.  Pins: the n = 1 closed form,
a family that decouples into 2 x 2 problems (``A = Q^H diag(a) Q``,
``B = Q^H diag(b) conj(Q)``), real data (where form II is form I), the
nonsymmetric eigensolver on ``H2``, the eigenvector relations, Lemma
ComputeNegEvecs part 2 and the closed-form eigenspace of a multiple eigenvalue;
a planted mistake must fail them.
"""
import numpy as np
import pytest

from oracle import bse as ob
from paper_2008_08825_amd import inputs


def sig(n):
    return np.concatenate([np.ones(n), -np.ones(n)])


def check_pairs(A, B, lam, X, tol=1e-12):
    n = A.shape[0]
    H = ob.bse_matrix_form2(A, B)
    scale = np.linalg.norm(H, 2)
    assert np.linalg.norm(H @ X - X * lam[None, :]) <= tol * scale * max(1.0, np.linalg.norm(X))
    G = X.conj().T @ (sig(n)[:, None] * X)
    assert np.abs(G - np.eye(n)).max() <= tol * 10


def decoupled_problem(n, seed):
    """A = Q^H diag(a) Q, B = Q^H diag(b) conj(Q) (complex symmetric), |b| < a:
    x_i = [Q^H e_i alpha; Q^T e_i beta] solves the 2 x 2 problem [[a, b], [-conj(b), -a]],
    so lambda_i = sqrt(a_i^2 - |b_i|^2)."""
    rng = np.random.default_rng(seed)
    Q = inputs.haar_unitary(rng, n)
    a = rng.uniform(1.0, 5.0, n)
    b = a * rng.uniform(0.0, 0.9, n) * np.exp(2j * np.pi * rng.uniform(size=n))
    A = Q.conj().T @ (a[:, None] * Q)
    A = (A + A.conj().T) / 2
    B = Q.conj().T @ (b[:, None] * Q.conj())
    B = (B + B.T) / 2
    return A, B, np.sort(np.sqrt(a * a - np.abs(b) ** 2))


def test_n1_closed_form():
    for a, b in [(2.0, 0.5 + 0.5j), (3.0, -1.2j), (1.0, 0.0), (5.0, 3.0 - 3.9j)]:
        A = np.array([[a]], complex)
        B = np.array([[b]], complex)
        lam, X = ob.solve_form2(A, B)
        assert abs(lam[0] - np.sqrt(a * a - abs(b) ** 2)) <= 1e-14 * a
        check_pairs(A, B, lam, X)


@pytest.mark.parametrize("n", [2, 7, 40])
def test_decoupled_closed_form(n):
    A, B, lref = decoupled_problem(n, seed=n)
    assert np.allclose(B, B.T)
    lam, X = ob.solve_form2(A, B)
    assert np.max(np.abs(lam - lref) / lref) <= 1e-13
    check_pairs(A, B, lam, X)


def test_real_data_is_form_one():
    A, B = inputs.coupled(30, seed=5)
    A, B = A.real.astype(complex), B.real.astype(complex)
    lam2, X2 = ob.solve_form2(A, B)
    lam1, _ = ob.solve_chol_svd(A, B)
    assert np.max(np.abs(lam2 - lam1) / lam1) <= 1e-13
    check_pairs(A, B, lam2, X2)


def test_dense_eig_and_negative_half():
    A, B, _ = decoupled_problem(9, seed=3)
    rng = np.random.default_rng(8)
    Z = rng.standard_normal((9, 9)) + 1j * rng.standard_normal((9, 9))
    A = A + 0.1 * (Z + Z.conj().T)          # a general (not decoupled) form-II matrix
    B = B + 0.05 * (Z + Z.T)
    lam, X = ob.solve_form2(A, B)
    w = np.linalg.eigvals(ob.bse_matrix_form2(A, B))
    assert np.max(np.abs(w.imag)) <= 1e-12 * np.max(np.abs(w))
    assert np.allclose(np.sort(w.real)[9:], lam, rtol=1e-12, atol=0)
    check_pairs(A, B, lam, X)
    lm, Y = ob.negative_half_form2(lam, X)
    H = ob.bse_matrix_form2(A, B)
    assert np.linalg.norm(H @ Y - Y * lm[None, :]) <= 1e-12 * np.linalg.norm(H, 2)
    assert np.abs(Y.conj().T @ (sig(9)[:, None] * Y) + np.eye(9)).max() <= 1e-11


def test_lower_triangle_inputs_only():
    A, B, lref = decoupled_problem(6, seed=11)
    Ag = np.tril(A) + np.triu(np.full_like(A, 7 + 7j), 1)
    Bg = np.tril(B) + np.triu(np.full_like(B, -3 + 1j), 1)
    Ag[np.diag_indices(6)] += 2j
    lam, _ = ob.solve_form2(Ag, Bg)
    assert np.max(np.abs(lam - lref) / lref) <= 1e-13


def test_planted_mistake_fails_the_pins(monkeypatch):
    """Hamiltonian with B in place of conj(B) (a plausible slip): the closed form catches it."""
    def wrong(A, B):
        A = ob.hermitian_from_lower(A)
        B = ob.symmetric_from_lower(B)
        return np.block([[A, B], [B, A.conj()]])
    monkeypatch.setattr(ob, "bse_hamiltonian_form2", wrong)
    A, B, lref = decoupled_problem(7, seed=7)
    try:
        lam, _ = ob.solve_form2(A, B)
        ok = lam.size == lref.size and np.max(np.abs(lam - lref) / lref) <= 1e-13
    except Exception:  # the wrong "Hamiltonian" is not Hermitian
        ok = False
    assert not ok


def test_multiple_eigenvalue_eigenspace():
    """A repeated (a_i, b_i) makes an eigenvalue of multiplicity 5; the oracle's vectors for it are
    Sigma-orthonormal and span the closed-form eigenspace {[Q^H e_i b_i; Q^T e_i (lambda - a_i)]}
    (each 2 x 2 block [[a, b], [-conj(b), -a]] has the eigenvector [b; lambda - a])."""
    n = 12
    rng = np.random.default_rng(4)
    Q = inputs.haar_unitary(rng, n)
    a = rng.uniform(1.0, 5.0, n)
    b = a * rng.uniform(0.1, 0.8, n) * np.exp(2j * np.pi * rng.uniform(size=n))
    run = np.arange(3, 8)
    a[run], b[run] = 2.0, 0.6 - 0.8j
    A = Q.conj().T @ (a[:, None] * Q)
    A = (A + A.conj().T) / 2
    B = Q.conj().T @ (b[:, None] * Q.conj())
    B = (B + B.T) / 2
    lam, X = ob.solve_form2(A, B)
    check_pairs(A, B, lam, X)
    lr = np.sqrt(2.0 ** 2 - abs(0.6 - 0.8j) ** 2)
    sel = np.abs(lam - lr) <= 1e-9 * lr
    assert sel.sum() == run.size
    E = np.eye(n)
    Xc = np.stack([np.concatenate([Q.conj().T @ E[:, i] * b[i], Q.T @ E[:, i] * (lr - a[i])]) for i in run], 1)
    Pc = Xc @ np.linalg.pinv(Xc)
    Xo = X[:, sel]
    Po = Xo @ np.linalg.pinv(Xo)
    assert np.linalg.norm(Pc - Po) <= 1e-12
