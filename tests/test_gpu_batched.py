"""Batched solve (grouped launches over problems of different orders) against the oracle.

Each problem of a batch must give what the oracle gives for it (same bars as
the single-problem parity tests), and exactly what bse_solve_h1 gives with the
same options and Jacobi tiles: a batch runs the same kernels on the same
per-problem arguments, only grouped into fewer launches.
"""
import numpy as np
import pytest
import torch

from oracle import bse as ob
from oracle import metrics as om
from paper_2008_08825_amd import inputs
from test_gpu_solver import check_against_oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(problems):
    As = [torch.from_numpy(A).to(DEV) for A, _ in problems]
    Bs = [torch.from_numpy(B).to(DEV) for _, B in problems]
    return As, Bs


def host(res):
    return [(lam.cpu().numpy(), X.resolve_conj().cpu().numpy()) for lam, X in res]


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_polish"])
def test_batched_uneven_sizes_vs_oracle(gpu_lib, precision):
    sizes = [130, 1, 65, 5, 200, 17, 64, 100, 3]
    problems = [inputs.coupled(n, seed=300 + i) for i, n in enumerate(sizes)]
    print(f"[gpu] batched {precision} sizes={sizes}", flush=True)
    res, infos, st = gpu_lib.solve_batched(*to_dev(problems), precision=precision, want_negative=True)
    assert st == 0 and all(i["status"] == 0 for i in infos)
    for (A, B), (lam, X), info in zip(problems, host(res), infos):
        n = A.shape[0]
        assert info["sweeps"] >= 1
        if precision != "mixed":
            check_against_oracle(A, B, lam, X)
        else:
            lam_o, _ = ob.solve_chol_svd(A, B)
            assert om.rel_eig_err(lam[:n], lam_o) < 1e-10
            assert om.residual(A, B, lam[:n], X[:, :n]) < 1e-13
        # negative half: eigenvalues -lambda, vectors [0 I; I 0] X
        assert np.array_equal(lam[n:], -lam[:n])
        assert np.array_equal(X[:n, n:], X[n:, :n]) and np.array_equal(X[n:, n:], X[:n, :n])


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_polish"])
def test_batched_equals_single_with_same_tiles(gpu_lib, precision):
    sizes = [130, 64, 200, 17, 256]
    tiles = [(64, 1, 64), (128, 2, 64), (192, 1, 64), (256, 4, 128)]
    problems = [inputs.coupled(n, seed=400 + i) for i, n in enumerate(sizes)]
    As, Bs = to_dev(problems)
    print(f"[gpu] batched vs single {precision}", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, Bs, precision=precision, tiles=tiles)
    assert st == 0
    for i, (lam_b, X_b) in enumerate(host(res)):
        lam, X, info = gpu_lib.solve_h1(As[i], Bs[i], precision=precision, tiles=tiles)
        assert np.array_equal(lam.cpu().numpy(), lam_b)
        assert np.array_equal(X.resolve_conj().cpu().numpy(), X_b)
        assert info["sweeps"] == infos[i]["sweeps"] and info["rotations"] == infos[i]["rotations"]
        if precision == "mixed_polish":
            assert info["polish_sweeps"] == infos[i]["polish_sweeps"] >= 1
            assert info["polish_rotations"] == infos[i]["polish_rotations"]
            assert info["max_off"] == infos[i]["max_off"] and infos[i]["fallback"] == 0


def test_batched_polish_fallback_branch(gpu_lib, monkeypatch):
    """The polished form's branch for a rotation that cannot be recovered (V'^H V' not
    positive definite; forced by the test hook), grouped: each problem's FP64 sweeps then
    run on W itself, bit for bit as the single solve's branch and as the FP64 form."""
    sizes = [130, 17, 200]
    tiles = [(64, 1, 64), (192, 1, 64), (256, 4, 128)]
    problems = [inputs.coupled(n, seed=450 + i) for i, n in enumerate(sizes)]
    As, Bs = to_dev(problems)
    monkeypatch.setenv("BSE_TEST_POLISH_FALLBACK", "1")
    print("[gpu] batched mixed_polish, forced fallback branch", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, Bs, precision="mixed_polish", tiles=tiles)
    assert st == 0 and all(i["fallback"] == 1 for i in infos)
    for i, (lam_b, X_b) in enumerate(host(res)):
        lam, X, info = gpu_lib.solve_h1(As[i], Bs[i], precision="mixed_polish", tiles=tiles)
        assert info["fallback"] == 1
        assert np.array_equal(lam.cpu().numpy(), lam_b)
        assert np.array_equal(X.resolve_conj().cpu().numpy(), X_b)
        lam64, X64, _ = gpu_lib.solve_h1(As[i], Bs[i], tiles=tiles)
        assert np.array_equal(lam64.cpu().numpy(), lam_b)
    monkeypatch.delenv("BSE_TEST_POLISH_FALLBACK")
    res2, infos2, st2 = gpu_lib.solve_batched(As, Bs, precision="mixed_polish", tiles=tiles)
    assert st2 == 0 and all(i["fallback"] == 0 for i in infos2)


def test_batched_mixed_windows_on_clustered_problems(gpu_lib):
    """Clustered spectra take the refinement's Rayleigh-Ritz window passes (grouped window
    eigensolvers and block GEMMs) in a batch: bit for bit the single solves' results (same
    tiles), the same window steps, and the oracle's eigenvalues."""
    # four tight clusters with weak coupling: at n ~ 1000 the complex64 start leaves pairs whose
    # first-order rotation exceeds 1/16 of their gap (what switches the windows on)
    sizes = [1024, 520, 300]
    tiles = [(320, 1, 64), (576, 1, 64), (1024, 4, 128)]
    problems = [inputs.clustered(n, seed=700 + i, clusters=4, width=1e-5, c_norm=1e-3, b_norm=1e-2)
                for i, n in enumerate(sizes)]
    As, Bs = to_dev(problems)
    print("[gpu] batched mixed, clustered problems", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, Bs, precision="mixed", tiles=tiles)
    assert st == 0
    assert any(i["refine_window_steps"] > 0 for i in infos), [i["refine_window_steps"] for i in infos]
    for i, (lam_b, X_b) in enumerate(host(res)):
        lam, X, info = gpu_lib.solve_h1(As[i], Bs[i], precision="mixed", tiles=tiles)
        assert np.array_equal(lam.cpu().numpy(), lam_b)
        assert np.array_equal(X.resolve_conj().cpu().numpy(), X_b)
        assert info["refine_window_steps"] == infos[i]["refine_window_steps"]
        assert info["refine_steps_done"] == infos[i]["refine_steps_done"]
        assert info["fallback"] == 0
        lam_o = ob.eigenvalues_chol_svd(*problems[i])
        assert om.rel_eig_err(lam_b, lam_o) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed_polish"])
def test_batched_status_per_problem(gpu_lib, precision):
    """One problem with A - B indefinite: its status is reported, the others are solved."""
    good = [inputs.coupled(n, seed=500 + n) for n in (40, 90)]
    A = np.diag(np.linspace(1.0, 2.0, 70)).astype(np.complex128)
    B = 0.5 * A
    B[30, 30] = 1.5 * A[30, 30]  # (A - B)[30, 30] < 0: leading minor 31 of A - B fails
    problems = [good[0], (A, B), good[1]]
    res, infos, st = gpu_lib.solve_batched(*to_dev(problems), precision=precision, check=False)
    assert st == 70 + 31 and infos[1]["status"] == 70 + 31 and infos[1]["fail_index"] == 31
    assert ob.chol_status(A, B) == 70 + 31
    assert infos[0]["status"] == 0 and infos[2]["status"] == 0
    out = host(res)
    for k in (0, 2):
        check_against_oracle(*problems[k], *out[k])


def test_batched_zero_sizes_and_empty(gpu_lib):
    res, infos, st = gpu_lib.solve_batched([], [])
    assert st == 0 and res == []
    A0 = torch.zeros((0, 0), dtype=torch.complex128, device=DEV)
    A, B = inputs.coupled(33, seed=7)
    res, infos, st = gpu_lib.solve_batched([A0, torch.from_numpy(A).to(DEV)], [A0, torch.from_numpy(B).to(DEV)])
    assert st == 0 and res[0][0].numel() == 0
    check_against_oracle(A, B, *host(res)[1:][0])


def test_batched_full_workload_256_problems(gpu_lib):
    """The 256-problem workload (n uniform in [64, 1024]), mixed form, as the benchmark runs it."""
    ns = inputs.batch_sizes()
    problems = [inputs.batch_problem(i, n) for i, n in enumerate(ns)]
    As, Bs = to_dev(problems)
    print("[gpu] batched 256-problem workload", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, Bs, precision="mixed")
    assert st == 0
    # properties at every size: Sigma-orthogonality and residual, on the GPU in FP64
    for i, ((lam, X), A, B) in enumerate(zip(res, As, Bs)):
        n = ns[i]
        X = X.resolve_conj()
        a, b = X[:n], X[n:]
        G = a.conj().T @ a - b.conj().T @ b
        orth = torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=DEV)).item()
        # residual of H1 = [A B; -B -A] scaled as the oracle's metric (Frobenius norms)
        R1 = A @ a + B @ b - a * lam
        R2 = -(B @ a) - A @ b - b * lam
        Hf = torch.sqrt(2 * torch.linalg.norm(A) ** 2 + 2 * torch.linalg.norm(B) ** 2)
        resid = (torch.sqrt(torch.linalg.norm(R1) ** 2 + torch.linalg.norm(R2) ** 2) / (Hf * torch.linalg.norm(X))).item()
        assert orth < 1e-9 * n ** 0.5 and resid < 1e-13, (i, n, orth, resid)
        assert infos[i]["refine_delta"] <= 1e-6
    # parity with the oracle on a sample: the three smallest problems, one near
    # 400 and the three largest (n close to 1024), eigenvalues and eigenvectors
    order = np.argsort(ns)
    sample = list(order[:3]) + [int(np.argmin(np.abs(np.array(ns) - 400)))] + list(order[-3:])
    for i in sample:
        A, B = problems[i]
        lam, X = res[i]
        lam = lam.cpu().numpy()
        X = X.resolve_conj().cpu().numpy()
        lam_o, X_o = ob.solve_chol_svd(A, B)
        assert om.rel_eig_err(lam, lam_o) < 1e-10, i
        err, gap = om.eigvec_errors(lam_o, X_o, X, cluster_rtol=1e-9)
        assert np.all(err <= 1e-10 + 1e-12 / np.minimum(gap, 1.0)), (i, ns[i], np.max(err))


def test_autotuner_small_range(gpu_lib):
    """The tuner picks valid tiles per bucket, and a batch solved with them matches the oracle."""
    from paper_2008_08825_amd import tune

    print("[gpu] autotuner np=64,128", flush=True)
    table, report = tune.tune(nps=(64, 128), precision="mixed", per_bucket=3, repeats=1)
    assert [r[0] for r in table] == [64, 128]
    for (np_, kc, rr) in table:
        assert (kc, rr) in tune.candidates(np_)
    sizes = [50, 128, 100, 64]
    problems = [inputs.coupled(n, seed=600 + n) for n in sizes]
    res, infos, st = gpu_lib.solve_batched(*to_dev(problems), precision="mixed", tiles=table)
    assert st == 0
    for (A, B), (lam, X) in zip(problems, host(res)):
        lam_o, _ = ob.solve_chol_svd(A, B)
        assert om.rel_eig_err(lam, lam_o) < 1e-10


def test_batched_alg2_equals_single_and_oracle(gpu_lib):
    """Alg. 2 (CHOL) in grouped launches: bit for bit the single solves (same tiles), the
    oracle's Alg. 2 pairs at the single tests' bars, the negative half, values only, and a
    problem with A + B indefinite reported while the others are solved."""
    sizes = [130, 1, 65, 200, 17]
    tiles = [(64, 1, 64), (192, 1, 64), (256, 4, 128)]
    problems = [inputs.coupled(n, seed=600 + i) for i, n in enumerate(sizes)]
    As, Bs = to_dev(problems)
    print("[gpu] batched alg2 vs single", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, Bs, route="eig", want_negative=True, tiles=tiles)
    assert st == 0
    out = host(res)
    for i, (lam_b, X_b) in enumerate(out):
        A, B = problems[i]
        n = A.shape[0]
        lam, X, info = gpu_lib.solve_h1(As[i], Bs[i], route="eig", want_negative=True, tiles=tiles)
        assert np.array_equal(lam.cpu().numpy(), lam_b)
        assert np.array_equal(X.resolve_conj().cpu().numpy(), X_b)
        assert info["sweeps"] == infos[i]["sweeps"] and info["rotations"] == infos[i]["rotations"]
        lam_o, X_o = ob.solve_chol_eig(A, B)
        assert om.rel_eig_err(lam_b[:n], lam_o) < 1e-11
        assert om.residual(A, B, lam_b[:n], X_b[:, :n]) < 1e-13
        err, gap = om.eigvec_errors(lam_o, X_o, X_b[:, :n], cluster_rtol=1e-9)
        assert np.all(err <= 1e-10 + 1e-13 / np.minimum(gap, 1.0))
        assert np.array_equal(lam_b[n:], -lam_b[:n])
    resv, _, stv = gpu_lib.solve_batched(As, Bs, route="eig", want_negative=True, tiles=tiles,
                                         values_only=True)
    assert stv == 0
    for (lam_v, _), (lam_b, _) in zip(resv, out):
        assert np.array_equal(lam_v.cpu().numpy(), lam_b)
    # A + B indefinite in the middle problem: status k (leading minor k of A + B)
    A, B = inputs.coupled(90, seed=61)
    B2 = B.copy()
    B2[40, 40] = A[40, 40].real + 1.0
    bad = [problems[0], (A, B2), problems[3]]
    res3, infos3, st3 = gpu_lib.solve_batched(*to_dev(bad), route="eig", check=False, tiles=tiles)
    assert st3 == ob.chol_status(A, B2) == infos3[1]["status"]
    assert infos3[0]["status"] == 0 and infos3[2]["status"] == 0
    assert np.array_equal(host(res3)[0][0], out[0][0][:sizes[0]])


def test_batched_tda_equals_single_and_oracle(gpu_lib):
    """Tamm-Dancoff batches (B = 0, Hermitian eigenproblem of A) in grouped launches: bit for
    bit the single solves (same tiles), the oracle's eigenpairs, values only."""
    sizes = [65, 1, 130, 2, 200]
    tiles = [(64, 1, 64), (192, 1, 64), (256, 4, 128)]
    As_h = [inputs.coupled(n, seed=620 + i)[0] for i, n in enumerate(sizes)]
    As = [torch.from_numpy(A).to(DEV) for A in As_h]
    print("[gpu] batched tda vs single", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, [None] * len(As), route="tda", want_negative=True, tiles=tiles)
    assert st == 0
    out = host(res)
    for i, (lam_b, X_b) in enumerate(out):
        n = sizes[i]
        lam, X, info = gpu_lib.solve_h1(As[i], None, route="tda", want_negative=True, tiles=tiles)
        assert np.array_equal(lam.cpu().numpy(), lam_b)
        assert np.array_equal(X.resolve_conj().cpu().numpy(), X_b)
        assert info["sweeps"] == infos[i]["sweeps"]
        lam_o, X_o = ob.solve_tda(As_h[i])
        assert om.rel_eig_err(lam_b[:n], lam_o) < 1e-13
        assert om.residual(As_h[i], np.zeros_like(As_h[i]), lam_b[:n], X_b[:, :n]) < 5e-14
        err, gap = om.eigvec_errors(lam_o, X_o, X_b[:, :n], cluster_rtol=1e-9)
        assert np.all(err <= 1e-11 + 1e-13 / np.minimum(gap, 1.0))
    resv, _, stv = gpu_lib.solve_batched(As, [None] * len(As), route="tda", want_negative=True,
                                         tiles=tiles, values_only=True)
    assert stv == 0
    for (lam_v, X_v), (lam_b, _) in zip(resv, out):
        assert X_v is None and np.array_equal(lam_v.cpu().numpy(), lam_b)


def test_batched_sqrt_route_equals_single_and_oracle(gpu_lib):
    """Alg. 1 (SQRT) batches in grouped launches (both Jacobi iterations, the k-scaled square
    root products): bit for bit the single solves (same tiles), the oracle's Alg. 1 pairs at
    the single test's bars, values only."""
    sizes = [130, 3, 65, 200]
    tiles = [(64, 1, 64), (192, 1, 64), (256, 4, 128)]
    problems = [inputs.coupled(n, seed=640 + i) for i, n in enumerate(sizes)]
    As, Bs = to_dev(problems)
    print("[gpu] batched sqrt route vs single", flush=True)
    res, infos, st = gpu_lib.solve_batched(As, Bs, route="sqrt", want_negative=True, tiles=tiles)
    assert st == 0
    out = host(res)
    for i, (lam_b, X_b) in enumerate(out):
        A, B = problems[i]
        n = A.shape[0]
        lam, X, info = gpu_lib.solve_h1(As[i], Bs[i], route="sqrt", want_negative=True, tiles=tiles)
        assert np.array_equal(lam.cpu().numpy(), lam_b)
        assert np.array_equal(X.resolve_conj().cpu().numpy(), X_b)
        assert info["sweeps"] == infos[i]["sweeps"] and info["rotations"] == infos[i]["rotations"]
        lam_o, X_o = ob.solve_sqrt(A, B)
        assert om.rel_eig_err(lam_b[:n], lam_o) < 1e-12
        assert om.residual(A, B, lam_b[:n], X_b[:, :n]) < 1e-13
        err, gap = om.eigvec_errors(lam_o, X_o, X_b[:, :n], cluster_rtol=1e-9)
        assert np.all(err <= 1e-10 + 1e-12 / np.minimum(gap, 1.0))
    resv, _, stv = gpu_lib.solve_batched(As, Bs, route="sqrt", want_negative=True, tiles=tiles,
                                         values_only=True)
    assert stv == 0
    for (lam_v, X_v), (lam_b, _) in zip(resv, out):
        assert X_v is None and np.array_equal(lam_v.cpu().numpy(), lam_b)
