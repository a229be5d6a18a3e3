"""Full-size parity: the n = 2048 workload in every form against the oracle's eigenvalues.

The oracle's eigenvalues come from tests/golden/oracle_n2048_eigenvalues.txt,
written by tests/golden/make_oracle_eigenvalues.py (oracle only).  Vectors at
this size are checked through properties that hold at any size: Sigma-
orthogonality and the residual of H1 X = X Lambda, computed on the GPU in FP64.
"""
import os

import numpy as np
import pytest
import torch

from paper_2008_08825_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_n2048_eigenvalues.txt")
# relative eigenvalue error gates: FP64 forms 1e-12, mixed form after refinement 1e-10
GATE = {"fp64": 1e-12, "mixed": 1e-10, "mixed_polish": 1e-12}


def sigma_orth_and_residual(A, B, lam, X):
    n = A.shape[0]
    a, b = X[:n], X[n:]
    G = a.mH @ a - b.mH @ b
    orth = torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=G.device)).item()
    R1 = A @ a + B @ b - a * lam
    R2 = -(B @ a) - A @ b - b * lam
    hn = torch.sqrt(2 * torch.linalg.norm(A) ** 2 + 2 * torch.linalg.norm(B) ** 2)
    res = (torch.sqrt(torch.linalg.norm(R1) ** 2 + torch.linalg.norm(R2) ** 2) / (hn * torch.linalg.norm(X))).item()
    return orth, res


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_polish"])
def test_n2048_workload_vs_oracle_eigenvalues(gpu_lib, precision):
    lam_o = np.loadtxt(GOLDEN)
    A_np, B_np = inputs.workload("n2048")
    n = A_np.shape[0]
    assert lam_o.shape == (n,)
    A = torch.from_numpy(A_np).to(DEV)
    B = torch.from_numpy(B_np).to(DEV)
    print(f"[gpu] n=2048 workload, {precision}", flush=True)
    lam, X, info = gpu_lib.solve_h1(A, B, precision=precision)
    rel = np.max(np.abs(lam.cpu().numpy() - lam_o) / lam_o)
    assert rel <= GATE[precision], rel
    orth, res = sigma_orth_and_residual(A, B, lam, X.resolve_conj())
    assert orth <= 1e-9 and res <= 1e-13, (orth, res)
