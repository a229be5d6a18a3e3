"""The entry point without allocation (bse_solve_h1_noalloc) against bse_solve_h1.

Two calls in a row on the same GPU, the second with a smaller order, so the
second runs in a scratch array that still holds the first call's data; each
must give the results of bse_solve_h1 with the same options (same kernels and
workspace plan, both Cholesky factorisations on the caller's stream: the
arithmetic is the same, so the outputs are compared bit for bit).
"""
import numpy as np
import pytest
import torch

from oracle import bse as ob
from oracle import metrics as om
from paper_2008_08825_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("precision", ["fp64", "mixed_polish", "mixed"])
def test_noalloc_matches_solve_h1(gpu_lib, precision):
    for n, seed in ((300, 31), (130, 32)):
        A, B = inputs.coupled(n, seed=seed)
        At = torch.from_numpy(A).to(DEV)
        Bt = torch.from_numpy(B).to(DEV)
        print(f"[gpu] noalloc n={n} {precision}", flush=True)
        lam0, X0, i0 = gpu_lib.solve_h1(At, Bt, precision=precision, want_negative=True)
        lam1, X1, i1 = gpu_lib.solve_h1_noalloc(At, Bt, precision=precision, want_negative=True)
        assert i1["status"] == 0
        lam0, lam1 = lam0.cpu().numpy(), lam1.cpu().numpy()
        X0, X1 = X0.resolve_conj().cpu().numpy(), X1.resolve_conj().cpu().numpy()
        assert np.array_equal(lam0, lam1) and np.array_equal(X0, X1)
        lam_o, _ = ob.solve_chol_svd(A, B)
        assert om.rel_eig_err(lam1[:n], lam_o) < (1e-10 if precision == "mixed" else 1e-12)
        assert om.residual(A, B, lam1[:n], X1[:, :n]) < 5e-14


def test_noalloc_rejects_orders_beyond_the_array(gpu_lib):
    cap = int(gpu_lib.load_library().bse_noalloc_scratch_bytes())
    assert cap == 64 << 20
    n = 1024
    assert gpu_lib.workspace_bytes(n) > cap
    A, B = inputs.coupled(n, seed=33)
    _, _, info = gpu_lib.solve_h1_noalloc(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV),
                                          check=False)
    assert info["status"] == -1
