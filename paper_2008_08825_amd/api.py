"""Python binding of the HIP solver's C ABI (``include/bse.h``).

Argument marshalling only: every step of the solve runs in ``libbse.so``.
PyTorch provides device memory (inputs, outputs, workspace) and the current
stream.  There is no CPU fallback; if the library is missing the calls raise.

Layout: torch tensors are row-major, the ABI is column-major.  A row-major
Hermitian ``A`` read as column-major is ``A^T = conj(A)``; the binding passes
row-major inputs with ``uplo='U'`` (which selects the lower triangle of the
row-major tensor), so the library solves the conjugated problem, whose
eigenvalues are the same and whose eigenvectors are the conjugates.  The
returned ``X`` is therefore a conjugated, transposed view of the library's
column-major buffer (no copy).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbse.so")

ROUTES = {"svd": 0, "eig": 1, "tda": 2, "sqrt": 3}
PRECISIONS = {"fp64": 0, "mixed": 1, "mixed_polish": 2}


class BSEOpts(ctypes.Structure):
    _fields_ = [
        ("route", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("max_sweeps", ctypes.c_int),
        ("refine_steps", ctypes.c_int),
        ("jacobi_tol", ctypes.c_double),
        ("want_negative", ctypes.c_int),
        ("uplo", ctypes.c_int),
        ("tile_entries", ctypes.c_int),
        ("checks", ctypes.c_int),
        ("tile_table", ctypes.POINTER(ctypes.c_int)),
        ("values_only", ctypes.c_int),
        ("reserved", ctypes.c_int),
    ]


class BSEInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("sweeps", ctypes.c_int),
        ("fail_index", ctypes.c_int),
        ("rotations", ctypes.c_int),
        ("max_off", ctypes.c_double),
        ("refine_delta", ctypes.c_double),
        ("ms_phase", ctypes.c_double * 8),
        ("timing", ctypes.c_int),
        ("pair_checks", ctypes.c_int),
        ("kernel_ms", ctypes.c_double * 3),
        ("kernel_launches", ctypes.c_int * 3),
        ("refine_steps_done", ctypes.c_int),
        ("inner_rotations", ctypes.c_double),
        ("polish_sweeps", ctypes.c_int),
        ("polish_rotations", ctypes.c_int),
        ("polish_pair_checks", ctypes.c_int),
        ("cross_pair_checks", ctypes.c_int),
        ("polish_max_off", ctypes.c_double),
        ("polish_inner_rotations", ctypes.c_double),
        ("polish_kernel_ms", ctypes.c_double * 3),
        ("polish_kernel_launches", ctypes.c_int * 3),
        ("polish_cross_pair_checks", ctypes.c_int),
        ("fallback", ctypes.c_int),
        ("sigma_orth_fro", ctypes.c_double),
        ("max_rel_resid", ctypes.c_double),
        ("refine_corr", ctypes.c_double * 8),
        ("refine_window_steps", ctypes.c_int),
    ]

    def as_dict(self):
        return {
            "status": self.status,
            "sweeps": self.sweeps,
            "fail_index": self.fail_index,
            "rotations": self.rotations,
            "max_off": self.max_off,
            "refine_delta": self.refine_delta,
            "ms_phase": list(self.ms_phase),
            "pair_checks": self.pair_checks,
            "cross_pair_checks": self.cross_pair_checks,
            "kernel_ms": list(self.kernel_ms),
            "kernel_launches": list(self.kernel_launches),
            "refine_steps_done": self.refine_steps_done,
            "inner_rotations": self.inner_rotations,
            "polish_sweeps": self.polish_sweeps,
            "polish_rotations": self.polish_rotations,
            "polish_pair_checks": self.polish_pair_checks,
            "polish_cross_pair_checks": self.polish_cross_pair_checks,
            "polish_max_off": self.polish_max_off,
            "polish_inner_rotations": self.polish_inner_rotations,
            "polish_kernel_ms": list(self.polish_kernel_ms),
            "polish_kernel_launches": list(self.polish_kernel_launches),
            "fallback": self.fallback,
            "sigma_orth_fro": self.sigma_orth_fro,
            "max_rel_resid": self.max_rel_resid,
            "refine_corr": list(self.refine_corr[: max(0, min(8, self.refine_steps_done))]),
            "refine_window_steps": self.refine_window_steps,
        }


PHASES = ["form", "chol", "W", "jacobi", "finalize", "back", "refine", "total"]

EXPORTS = [
    "bse_default_opts",
    "bse_workspace_bytes",
    "bse_solve_h1",
    "bse_batched_workspace_bytes",
    "bse_solve_batched",
    "bse_backward_workspace_bytes",
    "bse_backward",
    "bse_backward_vec_workspace_bytes",
    "bse_backward_vec",
    "bse_status_string",
    "bse_solve_h1_noalloc",
    "bse_noalloc_scratch_bytes",
    "bse_workspace_bytes_h2",
    "bse_solve_h2",
]

_lib = None


def load_library(path: Optional[str] = None):
    """Load ``libbse.so`` and declare the C signatures (raises if absent)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP solver library not built: {p} (run __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    ci = ctypes.c_int
    lib.bse_default_opts.argtypes = [ctypes.POINTER(BSEOpts)]
    lib.bse_default_opts.restype = None
    lib.bse_workspace_bytes.argtypes = [ci, ctypes.POINTER(BSEOpts)]
    lib.bse_workspace_bytes.restype = ctypes.c_size_t
    lib.bse_solve_h1.argtypes = [ci, vp, ci, vp, ci, vp, vp, ci, vp, ctypes.c_size_t,
                                 ctypes.POINTER(BSEOpts), ctypes.POINTER(BSEInfo), vp]
    lib.bse_solve_h1.restype = ci
    lib.bse_workspace_bytes_h2.argtypes = [ci, ctypes.POINTER(BSEOpts)]
    lib.bse_workspace_bytes_h2.restype = ctypes.c_size_t
    lib.bse_solve_h2.argtypes = [ci, vp, ci, vp, ci, vp, vp, ci, vp, ctypes.c_size_t,
                                 ctypes.POINTER(BSEOpts), ctypes.POINTER(BSEInfo), vp]
    lib.bse_solve_h2.restype = ci
    lib.bse_batched_workspace_bytes.argtypes = [ci, ctypes.POINTER(ci), ctypes.POINTER(BSEOpts)]
    lib.bse_batched_workspace_bytes.restype = ctypes.c_size_t
    lib.bse_solve_batched.argtypes = [ci, ctypes.POINTER(ci), ctypes.POINTER(vp), ctypes.POINTER(ci),
                                      ctypes.POINTER(vp), ctypes.POINTER(ci), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(ci), vp, ctypes.c_size_t,
                                      ctypes.POINTER(BSEOpts), ctypes.POINTER(BSEInfo), vp]
    lib.bse_solve_batched.restype = ci
    lib.bse_backward_workspace_bytes.argtypes = [ci]
    lib.bse_backward_workspace_bytes.restype = ctypes.c_size_t
    lib.bse_backward.argtypes = [ci, vp, ci, vp, vp, ci, vp, ci, vp, ctypes.c_size_t, vp]
    lib.bse_backward.restype = ci
    lib.bse_backward_vec_workspace_bytes.argtypes = [ci]
    lib.bse_backward_vec_workspace_bytes.restype = ctypes.c_size_t
    lib.bse_backward_vec.argtypes = [ci, vp, vp, ci, vp, vp, ci, ctypes.c_double, vp, ci, vp, ci, vp,
                                     ctypes.c_size_t, vp]
    lib.bse_backward_vec.restype = ci
    lib.bse_status_string.argtypes = [ci, ci]
    lib.bse_status_string.restype = ctypes.c_char_p
    lib.bse_solve_h1_noalloc.argtypes = [ci, vp, ci, vp, ci, vp, vp, ci, ctypes.POINTER(BSEOpts),
                                         ctypes.POINTER(BSEInfo), vp]
    lib.bse_solve_h1_noalloc.restype = ci
    lib.bse_noalloc_scratch_bytes.argtypes = []
    lib.bse_noalloc_scratch_bytes.restype = ctypes.c_size_t
    if path is None:
        _lib = lib
    return lib


class BSEError(RuntimeError):
    def __init__(self, status: int, n: int, info=None):
        lib = load_library()
        msg = lib.bse_status_string(status, n).decode()
        super().__init__(f"bse status {status}: {msg}")
        self.status = status
        self.info = info


def make_opts(route="svd", precision="fp64", max_sweeps=0, refine_steps=0, jacobi_tol=0.0,
              want_negative=False, uplo="L", tiles=None, checks=False, values_only=False) -> BSEOpts:
    """Options struct; ``tiles`` = rows ``(np_max, kc, rrows)`` of the Jacobi tile table."""
    o = BSEOpts()
    load_library().bse_default_opts(ctypes.byref(o))
    o.route = ROUTES[route]
    o.precision = PRECISIONS[precision]
    o.max_sweeps = int(max_sweeps)
    o.refine_steps = int(refine_steps)
    o.jacobi_tol = float(jacobi_tol)
    o.want_negative = 1 if want_negative else 0
    o.uplo = ord(uplo)
    o.checks = 1 if checks else 0
    o.values_only = 1 if values_only else 0
    if tiles:
        flat = [int(v) for row in tiles for v in row]
        arr = (ctypes.c_int * len(flat))(*flat)
        o._tiles_keep = arr  # the C side reads it during the call
        o.tile_table = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int))
        o.tile_entries = len(flat) // 3
    return o


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _matrix_arg(M: torch.Tensor, name: str):
    """(pointer, ld, uplo) for a square complex128 CUDA tensor, without copying when possible."""
    if M.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    if not M.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if M.dim() != 2 or M.shape[0] != M.shape[1]:
        raise ValueError(f"{name} must be square")
    if M.is_conj():
        M = M.resolve_conj()
    n = M.shape[0]
    if n == 0:
        return M, 0, 1, "L"
    if M.stride(1) == 1 and M.stride(0) >= max(1, n):
        # row-major: column-major view of A^T; its upper triangle is A's lower triangle
        return M, M.data_ptr(), M.stride(0), "U"
    if M.stride(0) == 1 and M.stride(1) >= max(1, n):
        return M, M.data_ptr(), M.stride(1), "L"
    M = M.contiguous()
    return M, M.data_ptr(), n, "U"


def workspace_bytes(n: int, **kw) -> int:
    lib = load_library()
    o = make_opts(**kw)
    return int(lib.bse_workspace_bytes(n, ctypes.byref(o)))


def solve_h1(A: torch.Tensor, B: Optional[torch.Tensor], *, route="svd", precision="fp64",
             want_negative=False, max_sweeps=0, refine_steps=0, jacobi_tol=0.0,
             timing=False, check=True, work: Optional[torch.Tensor] = None,
             out=None, tiles=None, checks=False, values_only=False):
    """All eigenpairs of H1 = [[A, B], [-B, -A]] (lower triangles of A, B read).

    Returns ``(lam, X, info)``: ``lam`` (n, ascending; 2n with ``want_negative``),
    ``X`` (2n x n or 2n x 2n, complex128) with ``H1 X = X diag(lam)`` and
    ``X^H Sigma X = I`` (``-I`` on the negative half), ``info`` a dict.
    ``route="tda"``: the Tamm-Dancoff approximation B = 0 (``B`` may be None).
    ``values_only``: eigenvalues alone, ``X`` is None.
    """
    lib = load_library()
    if B is None:
        if route != "tda":
            raise ValueError("B may be None only for route='tda'")
        B = A
    if A.shape != B.shape:
        raise ValueError("A and B must have the same shape")
    A_, pa, lda, ua = _matrix_arg(A, "A")
    B_, pb, ldb, ub = _matrix_arg(B, "B")
    if ua != ub:  # mixed layouts: bring B to A's
        B_ = B_.contiguous() if ua == "U" else B_.mT.contiguous().mT
        pb, ldb = B_.data_ptr(), (B_.stride(0) if ua == "U" else B_.stride(1))
    n = A.shape[0]
    dev = A.device
    ncols = 2 * n if want_negative else n
    o = make_opts(route, precision, max_sweeps, refine_steps, jacobi_tol, want_negative, ua, tiles,
                  checks, values_only)
    if out is None:
        lam = torch.empty(ncols, dtype=torch.float64, device=dev)
        Xbuf = None if values_only else torch.empty((ncols, 2 * n), dtype=torch.complex128, device=dev)
    else:
        lam, Xbuf = out
    need = int(lib.bse_workspace_bytes(n, ctypes.byref(o)))
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    info = BSEInfo()
    info.timing = int(timing)
    with torch.cuda.device(dev):
        st = lib.bse_solve_h1(n, pa, lda, pb, ldb, lam.data_ptr(),
                              Xbuf.data_ptr() if Xbuf is not None else None, max(1, 2 * n),
                              work.data_ptr(), work.numel(), ctypes.byref(o), ctypes.byref(info),
                              _stream_handle(dev))
    d = info.as_dict()
    d["status"] = st
    if check and st != 0:
        raise BSEError(st, n, d)
    if Xbuf is None:
        return lam, None, d
    X = Xbuf.mT
    if ua == "U":
        X = X.conj()
    return lam, X, d


def solve_h2(A: torch.Tensor, B: torch.Tensor, *, route="svd", precision="fp64", want_negative=False,
             max_sweeps=0, refine_steps=0, jacobi_tol=0.0, check=True,
             work: Optional[torch.Tensor] = None, tiles=None, values_only=False, checks=False):
    """All eigenpairs of a form-II matrix H2 = [[A, B], [-B^H, -A^T]] (A Hermitian,
    B complex symmetric; lower triangles read) through ``bse_solve_h2``.

    Returns ``(lam, X, info)`` as :func:`solve_h1`; the negative half is
    ``[[0, I], [I, 0]] conj(X)``.  ``checks`` fills ``info["sigma_orth_fro"]``
    (``|X^H Sigma X - I|_F``) and ``info["max_rel_resid"]`` on the device.
    """
    lib = load_library()
    if A.shape != B.shape or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A and B must be square and of the same shape")
    n = A.shape[0]
    dev = A.device
    # column-major copies: the transposed view of B is B itself but that of A is conj(A),
    # so the row-major trick of solve_h1 does not apply to form II
    Ac = A.to(torch.complex128).mT.contiguous()
    Bc = B.to(torch.complex128).mT.contiguous()
    ncols = 2 * n if want_negative else n
    o = make_opts(route, precision, max_sweeps, refine_steps, jacobi_tol, want_negative, "L", tiles,
                  checks, values_only)
    lam = torch.empty(ncols, dtype=torch.float64, device=dev)
    Xbuf = None if values_only else torch.empty((ncols, 2 * n), dtype=torch.complex128, device=dev)
    need = int(lib.bse_workspace_bytes_h2(n, ctypes.byref(o)))
    if need == 0 and n > 0:
        raise ValueError("invalid order or options for form II")
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    info = BSEInfo()
    with torch.cuda.device(dev):
        st = lib.bse_solve_h2(n, Ac.data_ptr(), max(1, n), Bc.data_ptr(), max(1, n), lam.data_ptr(),
                              Xbuf.data_ptr() if Xbuf is not None else None, max(1, 2 * n),
                              work.data_ptr(), work.numel(), ctypes.byref(o), ctypes.byref(info),
                              _stream_handle(dev))
    d = info.as_dict()
    d["status"] = st
    if check and st != 0:
        raise BSEError(st, 2 * n, d)
    return lam, (None if Xbuf is None else Xbuf.mT), d


def solve_h1_noalloc(A: torch.Tensor, B: torch.Tensor, *, route="svd", precision="fp64",
                     want_negative=False, max_sweeps=0, refine_steps=0, jacobi_tol=0.0,
                     check=True, out=None, checks=False):
    """:func:`solve_h1` through ``bse_solve_h1_noalloc``: the library's own
    per-GPU scratch array instead of a workspace (no device allocation in the
    call; ``out`` = preallocated ``(lam, Xbuf)`` avoids torch's as well).
    Orders whose workspace exceeds the array return status -1."""
    lib = load_library()
    if A.shape != B.shape:
        raise ValueError("A and B must have the same shape")
    A_, pa, lda, ua = _matrix_arg(A, "A")
    B_, pb, ldb, ub = _matrix_arg(B, "B")
    if ua != ub:
        B_ = B_.contiguous() if ua == "U" else B_.mT.contiguous().mT
        pb, ldb = B_.data_ptr(), (B_.stride(0) if ua == "U" else B_.stride(1))
    n = A.shape[0]
    dev = A.device
    ncols = 2 * n if want_negative else n
    o = make_opts(route, precision, max_sweeps, refine_steps, jacobi_tol, want_negative, ua, None,
                  checks)
    if out is None:
        lam = torch.empty(ncols, dtype=torch.float64, device=dev)
        Xbuf = torch.empty((ncols, 2 * n), dtype=torch.complex128, device=dev)
    else:
        lam, Xbuf = out
    info = BSEInfo()
    with torch.cuda.device(dev):
        st = lib.bse_solve_h1_noalloc(n, pa, lda, pb, ldb, lam.data_ptr(), Xbuf.data_ptr(),
                                      max(1, 2 * n), ctypes.byref(o), ctypes.byref(info),
                                      _stream_handle(dev))
    d = info.as_dict()
    d["status"] = st
    if check and st != 0:
        raise BSEError(st, n, d)
    X = Xbuf.mT
    if ua == "U":
        X = X.conj()
    return lam, X, d


def solve_batched(As, Bs, *, route="svd", precision="fp64", want_negative=False,
                  max_sweeps=0, refine_steps=0, jacobi_tol=0.0, check=True, tiles=None,
                  timing=0, work=None, values_only=False):
    """Independent problems ``(A_i, B_i)`` in one library call; returns lists of (lam, X) and infos.

    ``tiles``: rows ``(np_max, kc, rrows)`` of the Jacobi tile table (see
    :mod:`paper_2008_08825_amd.tune`); ``work``: optional preallocated uint8
    CUDA workspace of at least ``batched_workspace_bytes`` bytes.
    """
    lib = load_library()
    count = len(As)
    if len(Bs) != count:
        raise ValueError("As and Bs differ in length")
    keep = []
    ns, pas, ldas, pbs, ldbs, plams, pxs, ldxs, uplos = [], [], [], [], [], [], [], [], []
    lams, Xbufs = [], []
    dev = As[0].device if count else torch.device("cuda")
    for A, B in zip(As, Bs):
        if B is None:  # route "tda": B is not read
            if route != "tda":
                raise ValueError("B may be None only for route='tda'")
            B = A
        A_, pa, lda, ua = _matrix_arg(A, "A")
        B_, pb, ldb, ub = _matrix_arg(B, "B")
        if ua != "U" or ub != "U":
            A_ = A_.contiguous() if ua != "U" else A_
            B_ = B_.contiguous() if ub != "U" else B_
            pa, lda, pb, ldb = A_.data_ptr(), A_.stride(0), B_.data_ptr(), B_.stride(0)
        keep += [A_, B_]
        n = A.shape[0]
        ncols = 2 * n if want_negative else n
        lam = torch.empty(ncols, dtype=torch.float64, device=dev)
        Xb = None if values_only else torch.empty((ncols, 2 * n), dtype=torch.complex128, device=dev)
        lams.append(lam)
        Xbufs.append(Xb)
        ns.append(n); pas.append(pa); ldas.append(max(1, lda)); pbs.append(pb); ldbs.append(max(1, ldb))
        plams.append(lam.data_ptr()); pxs.append(Xb.data_ptr() if Xb is not None else None)
        ldxs.append(max(1, 2 * n))
    o = make_opts(route, precision, max_sweeps, refine_steps, jacobi_tol, want_negative, "U", tiles,
                  False, values_only)
    IA = ctypes.c_int * max(count, 1)
    PA = ctypes.c_void_p * max(count, 1)
    c_n = IA(*ns)
    need = int(lib.bse_batched_workspace_bytes(count, c_n, ctypes.byref(o)))
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    infos = (BSEInfo * max(count, 1))()
    if count:
        infos[0].timing = int(timing)
    with torch.cuda.device(dev):
        st = lib.bse_solve_batched(count, c_n, PA(*pas), IA(*ldas), PA(*pbs), IA(*ldbs), PA(*plams),
                                   PA(*pxs), IA(*ldxs), work.data_ptr(), work.numel(), ctypes.byref(o),
                                   infos, _stream_handle(dev))
    out_infos = [infos[i].as_dict() for i in range(count)]
    if check and st != 0:
        raise BSEError(st, ns[0] if ns else 0, out_infos)
    results = [(lams[i], None if values_only else Xbufs[i].mT.conj()) for i in range(count)]
    return results, out_infos, st


def batched_workspace_bytes(ns, *, route="svd", precision="fp64", tiles=None, values_only=False) -> int:
    lib = load_library()
    o = make_opts(route, precision, tiles=tiles, values_only=values_only)
    IA = ctypes.c_int * max(len(ns), 1)
    return int(lib.bse_batched_workspace_bytes(len(ns), IA(*[int(v) for v in ns]), ctypes.byref(o)))


def backward(X: torch.Tensor, w: torch.Tensor):
    """``(G_A, G_B)`` for ``L = sum_k w_k lambda_k`` (see ``bse_backward`` in include/bse.h)."""
    lib = load_library()
    n2, n = X.shape
    if n2 != 2 * n:
        raise ValueError("X must be 2n x n")
    if X.dtype != torch.complex128 or not X.is_cuda:
        raise TypeError("X must be a complex128 CUDA tensor")
    w = w.to(dtype=torch.float64, device=X.device).contiguous()
    conj = X.is_conj()
    Xr = X.conj() if conj else X            # buffer values (conj bit dropped, no copy)
    Xr = Xr.resolve_conj()
    if Xr.stride(0) != 1 or Xr.stride(1) < max(1, 2 * n):
        Xr = Xr.mT.contiguous().mT
    dev = X.device
    gA = torch.empty((n, n), dtype=torch.complex128, device=dev)
    gB = torch.empty((n, n), dtype=torch.complex128, device=dev)
    work = torch.empty(max(1, int(lib.bse_backward_workspace_bytes(n))), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        st = lib.bse_backward(n, Xr.data_ptr(), Xr.stride(1), w.data_ptr(), gA.data_ptr(), n,
                              gB.data_ptr(), n, work.data_ptr(), work.numel(), _stream_handle(dev))
    if st != 0:
        raise BSEError(st, n)
    # gA, gB hold column-major G computed from the buffer values; the row-major
    # reading of that memory is G^T, and conjugated inputs give conj(G).
    GA = gA.mT
    GB = gB.mT
    if conj:
        GA = GA.conj()
        GB = GB.conj()
    return GA, GB


def _colmajor(M: torch.Tensor, rows: int) -> torch.Tensor:
    """``M`` (rows x cols) or a copy whose memory is column-major with leading dimension >= rows.

    The copy goes through an explicit (cols, rows) buffer: torch ignores the
    stride of a dimension of size 1, so ``.mT.contiguous()`` may keep one."""
    if M.stride(0) != 1 or M.stride(1) < max(1, rows):
        buf = torch.empty((M.shape[1], M.shape[0]), dtype=M.dtype, device=M.device)
        buf.copy_(M.mT)
        M = buf.mT
    return M


def backward_vec(lam: torch.Tensor, X: torch.Tensor, g_lam: Optional[torch.Tensor],
                 G_X: Optional[torch.Tensor], degen_rtol: float = 1e-13):
    """``(G_A, G_B)`` for a loss of the eigenvalues and eigenvectors (``bse_backward_vec``).

    ``lam`` (n) and ``X`` (2n x n) as returned by :func:`solve_h1`; ``g_lam``
    = dL/dlam and ``G_X`` the gradient with respect to ``X`` (PyTorch's
    convention for complex tensors); either may be None (zero).
    """
    lib = load_library()
    n2, n = X.shape
    if n2 != 2 * n:
        raise ValueError("X must be 2n x n")
    if X.dtype != torch.complex128 or not X.is_cuda:
        raise TypeError("X must be a complex128 CUDA tensor")
    dev = X.device
    lam = lam[:n].to(dtype=torch.float64, device=dev).contiguous()
    g = (torch.zeros(n, dtype=torch.float64, device=dev) if g_lam is None
         else g_lam[:n].to(dtype=torch.float64, device=dev).contiguous())
    conj = X.is_conj()
    # buffer values: for a conjugated view the library sees conj(X) and, with
    # Re tr(G^H conj(dX)) = Re tr(conj(G)^H dX), the gradient conj(G_X)
    Xr = _colmajor((X.conj() if conj else X).resolve_conj(), 2 * n)
    if G_X is None:
        G = torch.zeros((2 * n, n), dtype=torch.complex128, device=dev)
    else:
        G = G_X.to(dtype=torch.complex128, device=dev)
        G = G.conj() if conj else G
    Gr = _colmajor(G.resolve_conj(), 2 * n)
    gA = torch.empty((n, n), dtype=torch.complex128, device=dev)
    gB = torch.empty((n, n), dtype=torch.complex128, device=dev)
    work = torch.empty(max(1, int(lib.bse_backward_vec_workspace_bytes(n))), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        st = lib.bse_backward_vec(n, lam.data_ptr(), Xr.data_ptr(), Xr.stride(1), g.data_ptr(),
                                  Gr.data_ptr(), Gr.stride(1), float(degen_rtol), gA.data_ptr(), n,
                                  gB.data_ptr(), n, work.data_ptr(), work.numel(), _stream_handle(dev))
    if st != 0:
        raise BSEError(st, n)
    GA = gA.mT
    GB = gB.mT
    if conj:
        GA = GA.conj()
        GB = GB.conj()
    return GA, GB


class BSEEig(torch.autograd.Function):
    """``(lam, X) = BSEEig.apply(A, B)``, differentiable through ``lam`` and ``X``.

    The gradient is the full Hermitian ``G`` with ``dL = Re tr(G^H dA)`` for
    Hermitian perturbations.  Losses of the eigenvalues alone take
    ``bse_backward``; a loss that also depends on ``X`` takes
    ``bse_backward_vec`` (it should not depend on the phase of each column).
    """

    @staticmethod
    def forward(ctx, A, B, route="svd", precision="fp64"):
        lam, X, _ = solve_h1(A.detach(), B.detach(), route=route, precision=precision)
        ctx.save_for_backward(lam, X)
        return lam, X

    @staticmethod
    def backward(ctx, g_lam, g_X):
        lam, X = ctx.saved_tensors
        if g_X is not None and bool(torch.any(g_X != 0)):
            GA, GB = backward_vec(lam, X, g_lam, g_X)
            return GA, GB, None, None
        if g_lam is None:
            return None, None, None, None
        GA, GB = backward(X, g_lam)
        return GA, GB, None, None
