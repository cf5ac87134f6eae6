"""Python binding of libtchol (tiled FP64 Cholesky on one MI355X).

Argument marshalling only: every step of the factorization and of the solve
runs in the library's HIP kernels; torch provides device memory and the
stream.  There is no CPU fallback: if libtchol.so has not been built, or no
GPU is visible, the calls raise.

Layout.  torch tensors are row-major.  The library works on column-major
storage and reads only the lower triangle.  A symmetric row-major A has the
same bytes as its column-major self, so it is passed unchanged; after the
factorization its column-major lower triangle holds L, i.e. the row-major
view holds L^T in its upper triangle and ``A.mT`` is L (lower part).
Right-hand sides are passed as a column-major copy (``B.mT.contiguous()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtchol.so")

OP_FACTOR, OP_SOLVE, OP_BATCHED, OP_BACKWARD, OP_MIXED_FACTOR, OP_FACTOR_SOLVE = 0, 1, 2, 3, 4, 5
POLICY_LIST, POLICY_RANK, POLICY_FIFO, POLICY_RANDOM = 0, 1, 2, 3
E_HIP, E_TIMEOUT, E_UNSUPPORTED, E_INTERNAL, E_NOCONV, E_SCRATCH = -100, -101, -102, -103, -104, -105
NOALLOC_SCRATCH_BYTES = 16 << 20
LOWP_FP32, LOWP_BF16 = 1, 2
KIND_NAMES = ["POTRF", "TRSM", "SYRK", "GEMM", "FTRSV", "FGEMV", "BTRSV", "BGEMV", "GREV", "TREV", "DPART", "PREV",
              "TRTRI", "DRED", "GEMM2", "PADJM", "PADJY", "PADJS",
              "GREV2"]

_lib = None


class TcholError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %d (%s)" % (where, code, strerror(code) if _lib else "?"))


class Opts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("seed", ctypes.c_uint32), ("wait_limit_us", ctypes.c_int64),
                ("kernel_ms", ctypes.POINTER(ctypes.c_float)), ("trace", ctypes.c_void_p),
                ("trace_words", ctypes.c_int64), ("subst", ctypes.c_int32),
                ("wgs", ctypes.POINTER(ctypes.c_int32)), ("inv_trsm", ctypes.c_int32)]


def load() -> ctypes.CDLL:
    """Load libtchol.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtchol.so is not built; run `python -m paper_1402_6601_amd.build` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
    P32 = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    lib.tchol_workspace_bytes.restype = i64
    lib.tchol_workspace_bytes.argtypes = [i32, i64, i64, i64]
    lib.tchol_factor.restype = i32
    lib.tchol_factor.argtypes = [vp, i64, i64, vp, i64, vp]
    lib.tchol_factor_ex.restype = i32
    lib.tchol_factor_ex.argtypes = [vp, i64, i64, vp, i64, vp, ctypes.POINTER(Opts)]
    lib.tchol_solve.restype = i32
    lib.tchol_solve.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp]
    lib.tchol_solve_ex.restype = i32
    lib.tchol_solve_ex.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, ctypes.POINTER(Opts)]
    lib.tchol_backward.restype = i32
    lib.tchol_backward.argtypes = [vp, i64, i64, vp, vp, i64, vp]
    lib.tchol_backward_ex.restype = i32
    lib.tchol_backward_ex.argtypes = [vp, i64, i64, vp, vp, i64, vp, ctypes.POINTER(Opts)]
    lib.tchol_mixed_workspace_bytes.restype = i64
    lib.tchol_mixed_workspace_bytes.argtypes = [i64, i64, i64]
    lib.tchol_mixed_workspace_bytes_ex.restype = i64
    lib.tchol_mixed_workspace_bytes_ex.argtypes = [i64, i64, i64, i32]
    lib.tchol_solve_mixed.restype = i32
    lib.tchol_solve_mixed.argtypes = [vp, i64, i64, vp, i64, i32, ctypes.c_double, i32,
                                      ctypes.POINTER(ctypes.c_double), P32, vp, i64, vp, ctypes.POINTER(Opts)]
    lib.tchol_strerror.restype = ctypes.c_char_p
    lib.tchol_strerror.argtypes = [i32]
    lib.tchol_version.restype = ctypes.c_char_p
    lib.tchol_version.argtypes = []
    lib.tchol_plan_query.restype = i32
    lib.tchol_plan_query.argtypes = [i32, i64, i64, i32, u32, P64, P32, P32, P32, P32, P32, P32, P64, P32, P32,
                                     P32, P32]
    lib.tchol_batched_plan_query.restype = i32
    lib.tchol_batched_plan_query.argtypes = [P32, P32, i32, i32, u32, P32, P64, P32, P32, P32, P32, P32, P32, P32, P64,
                                             P32, P32, P32, P32]
    lib.tchol_batched_workspace_bytes.restype = i64
    lib.tchol_batched_workspace_bytes.argtypes = [P32, P32, i32]
    lib.tchol_factor_solve_workspace_bytes.restype = i64
    lib.tchol_factor_solve_workspace_bytes.argtypes = [i64, i64, i64]
    lib.tchol_factor_solve.restype = i32
    lib.tchol_factor_solve.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, ctypes.POINTER(Opts)]
    lib.tchol_factor_solve_noalloc.restype = i32
    lib.tchol_factor_solve_noalloc.argtypes = [vp, i64, i64, vp, i64, vp]
    lib.tchol_batched_f32_workspace_bytes.restype = i64
    lib.tchol_batched_f32_workspace_bytes.argtypes = [P32, P32, i32, i32]
    lib.tchol_factor_solve_batched_f32.restype = i32
    lib.tchol_factor_solve_batched_f32.argtypes = [vp, P64, P32, vp, P64, P32, P32, i32, i32, P32, vp, i64, vp,
                                                   ctypes.POINTER(Opts)]
    lib.tchol_factor_solve_batched.restype = i32
    lib.tchol_factor_solve_batched.argtypes = [vp, P64, P32, vp, P64, P32, P32, i32, i32, P32, vp, i64, vp,
                                               ctypes.POINTER(Opts)]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().tchol_strerror(int(code)).decode()


def version() -> str:
    return load().tchol_version().decode()


def workspace_bytes(op: int, n: int, nb: int, nrhs: int = 0) -> int:
    r = load().tchol_workspace_bytes(op, n, nb, nrhs)
    if r < 0:
        raise TcholError(int(r), "tchol_workspace_bytes")
    return int(r)


def factor_solve_workspace_bytes(n: int, nb: int, nrhs: int) -> int:
    """Bytes of workspace of the merged factor + solve launch (tchol_factor_solve)."""
    r = load().tchol_factor_solve_workspace_bytes(n, nb, nrhs)
    if r < 0:
        raise TcholError(int(r), "tchol_factor_solve_workspace_bytes")
    return int(r)


# ---------------------------------------------------------------- plan introspection (host only)

def plan_query(op: int, n: int, nb: int, policy: int = POLICY_LIST, seed: int = 0) -> dict:
    """The task DAG, ranks and claim order the library would execute (no GPU needed)."""
    lib = load()
    counts = np.zeros(4, dtype=np.int64)
    P32 = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    null32, null64 = ctypes.cast(None, P32), ctypes.cast(None, P64)
    rc = lib.tchol_plan_query(op, n, nb, policy, seed, counts.ctypes.data_as(P64), null32, null32, null32, null32,
                              null32, null32, null64, null32, null32, null32, null32)
    if rc != 0:
        raise TcholError(rc, "tchol_plan_query")
    nt, ne, ni = int(counts[0]), int(counts[1]), int(counts[2])
    a = {k: np.zeros(nt, dtype=np.int32) for k in ("kind", "i", "j", "k", "parts", "dep0")}
    a["rank"] = np.zeros(nt, dtype=np.int64)
    a["succ_off"] = np.zeros(nt + 1, dtype=np.int32)
    a["succ"] = np.zeros(max(ne, 1), dtype=np.int32)
    a["item_task"] = np.zeros(max(ni, 1), dtype=np.int32)
    a["item_part"] = np.zeros(max(ni, 1), dtype=np.int32)
    p = lambda x: x.ctypes.data_as(P32)
    rc = lib.tchol_plan_query(op, n, nb, policy, seed, counts.ctypes.data_as(P64), p(a["kind"]), p(a["i"]),
                              p(a["j"]), p(a["k"]), p(a["parts"]), p(a["dep0"]), a["rank"].ctypes.data_as(P64),
                              p(a["succ_off"]), p(a["succ"]), p(a["item_task"]), p(a["item_part"]))
    if rc != 0:
        raise TcholError(rc, "tchol_plan_query")
    a["succ"] = a["succ"][:ne]
    a["item_task"] = a["item_task"][:ni]
    a["item_part"] = a["item_part"][:ni]
    a["ntask"], a["nedge"], a["nitem"], a["critical_path"] = nt, ne, ni, int(counts[3])
    return a


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def batched_plan_query(n, nb, policy: int = POLICY_LIST, seed: int = 0, wgs=None) -> dict:
    """The merged factor + solve DAG of a batched launch (no GPU needed); as
    plan_query, plus "sys", the system of every task.  wgs as for
    factor_solve_batched_."""
    lib = load()
    n32, nb32 = _i32(n), _i32(nb)
    w32 = None if wgs is None else _i32(wgs)
    if w32 is not None and len(w32) != len(n32):
        raise ValueError("wgs must have one entry per system")
    P32 = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    null32, null64 = ctypes.cast(None, P32), ctypes.cast(None, P64)
    counts = np.zeros(4, dtype=np.int64)
    p = lambda x: x.ctypes.data_as(P32)
    pw = null32 if w32 is None else p(w32)
    rc = lib.tchol_batched_plan_query(p(n32), p(nb32), len(n32), policy, seed, pw, counts.ctypes.data_as(P64),
                                      null32, null32, null32, null32, null32, null32, null32, null64, null32,
                                      null32, null32, null32)
    if rc != 0:
        raise TcholError(rc, "tchol_batched_plan_query")
    nt, ne, ni = int(counts[0]), int(counts[1]), int(counts[2])
    a = {k: np.zeros(max(nt, 1), dtype=np.int32) for k in ("kind", "i", "j", "k", "sys", "parts", "dep0")}
    a["rank"] = np.zeros(max(nt, 1), dtype=np.int64)
    a["succ_off"] = np.zeros(nt + 1, dtype=np.int32)
    a["succ"] = np.zeros(max(ne, 1), dtype=np.int32)
    a["item_task"] = np.zeros(max(ni, 1), dtype=np.int32)
    a["item_part"] = np.zeros(max(ni, 1), dtype=np.int32)
    rc = lib.tchol_batched_plan_query(p(n32), p(nb32), len(n32), policy, seed, pw, counts.ctypes.data_as(P64),
                                      p(a["kind"]), p(a["i"]), p(a["j"]), p(a["k"]), p(a["sys"]), p(a["parts"]),
                                      p(a["dep0"]), a["rank"].ctypes.data_as(P64), p(a["succ_off"]), p(a["succ"]),
                                      p(a["item_task"]), p(a["item_part"]))
    if rc != 0:
        raise TcholError(rc, "tchol_batched_plan_query")
    for k in ("kind", "i", "j", "k", "sys", "parts", "dep0", "rank"):
        a[k] = a[k][:nt]
    a["succ"] = a["succ"][:ne]
    a["item_task"] = a["item_task"][:ni]
    a["item_part"] = a["item_part"][:ni]
    a["ntask"], a["nedge"], a["nitem"], a["critical_path"] = nt, ne, ni, int(counts[3])
    return a


def mixed_workspace_bytes(n: int, nb: int, nrhs: int, lowp: int = LOWP_FP32) -> int:
    r = load().tchol_mixed_workspace_bytes_ex(n, nb, nrhs, lowp)
    if r < 0:
        raise TcholError(int(r), "tchol_mixed_workspace_bytes_ex")
    return int(r)


def batched_workspace_bytes(n, nb) -> int:
    n32, nb32 = _i32(n), _i32(nb)
    P32 = ctypes.POINTER(ctypes.c_int32)
    r = load().tchol_batched_workspace_bytes(n32.ctypes.data_as(P32), nb32.ctypes.data_as(P32), len(n32))
    if r < 0:
        raise TcholError(int(r), "tchol_batched_workspace_bytes")
    return int(r)


# ---------------------------------------------------------------- device entry points

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("tchol needs a ROCm GPU; none is visible")
    return torch


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(torch, nbytes: int, device):
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return ws


def _opts(policy, seed, wait_limit_us, want_ms, trace, subst=False):
    o = Opts()
    o.policy = policy
    o.seed = seed
    o.wait_limit_us = wait_limit_us
    o.subst = 1 if subst else 0
    ms = ctypes.c_float(0.0)
    o.kernel_ms = ctypes.pointer(ms) if want_ms else ctypes.cast(None, ctypes.POINTER(ctypes.c_float))
    if trace is not None:
        if trace.element_size() != 8 or not trace.is_contiguous():
            raise ValueError("trace must be a contiguous tensor of 64-bit words")
        o.trace = ctypes.c_void_p(trace.data_ptr())
        o.trace_words = trace.numel()
    else:
        o.trace = None
        o.trace_words = 0
    return o, ms


def factor_(A, nb: int, *, policy: int = POLICY_LIST, seed: int = 0, wait_limit_us: int = 0, ws=None,
            want_kernel_ms: bool = False, trace=None, check: bool = True, inv_trsm: bool = False):
    """Factor in place.  A: CUDA float64 (n, n) contiguous, symmetric (only the
    lower triangle of its column-major reading, i.e. the row-major upper
    triangle, is read).  inv_trsm: TRSMs through the diagonal tiles' explicit
    inverses, as in factor_solve_ (tchol_opts.inv_trsm).  Returns info
    (0 = success), or (info, kernel_ms)."""
    torch = _torch()
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("A must be a contiguous square float64 tensor")
    if not A.is_cuda:
        raise ValueError("A must be on the GPU")
    n = A.shape[0]
    lib = load()
    with torch.cuda.device(A.device):
        need = workspace_bytes(OP_FACTOR, n, nb) if n else 256
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, A.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace)
        o.inv_trsm = 1 if inv_trsm else 0
        rc = lib.tchol_factor_ex(ctypes.c_void_p(A.data_ptr()), n, nb, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream_ptr(torch, A.device), ctypes.byref(o))
    if rc < 0 and check:
        raise TcholError(rc, "tchol_factor")
    return (rc, ms.value) if want_kernel_ms else rc


def factor(A, nb: int, **kw):
    """Return (L, info): L is the lower Cholesky factor of the symmetric A (a new tensor)."""
    torch = _torch()
    W = A.detach().to(dtype=torch.float64).contiguous().clone()
    info = factor_(W, nb, **kw)
    if isinstance(info, tuple):
        info = info[0]
    return torch.tril(W.mT), info


def solve_(L, Bc, nb: int, *, policy: int = POLICY_LIST, seed: int = 0, wait_limit_us: int = 0, ws=None,
           want_kernel_ms: bool = False, trace=None, check: bool = True, subst: bool = False):
    """Solve in place.  L: the (n, n) buffer factored by factor_ (column-major
    lower = L).  Bc: CUDA float64 (nrhs, n) contiguous, i.e. B column-major.
    trace: optional CUDA int64 tensor of 4 words per work item (see factor_).
    subst: substitute against the diagonal tiles instead of applying their
    explicit inverses (tchol_opts.subst)."""
    torch = _torch()
    n = L.shape[0]
    if Bc.dtype != torch.float64 or not Bc.is_contiguous() or Bc.dim() != 2 or Bc.shape[1] != n:
        raise ValueError("Bc must be a contiguous float64 (nrhs, n) tensor (B in column-major order)")
    nrhs = Bc.shape[0]
    lib = load()
    with torch.cuda.device(L.device):
        need = workspace_bytes(OP_SOLVE, n, nb, nrhs) if n else 256
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, L.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace, subst)
        rc = lib.tchol_solve_ex(ctypes.c_void_p(L.data_ptr()), n, nb, ctypes.c_void_p(Bc.data_ptr()), nrhs,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(torch, L.device),
                                ctypes.byref(o))
    if rc != 0 and check:
        raise TcholError(rc, "tchol_solve")
    return (rc, ms.value) if want_kernel_ms else rc


def solve(Lbuf, B, nb: int, **kw):
    """X = A^{-1} B given the factored buffer of factor_; B is (n,) or (n, nrhs)."""
    vec = B.dim() == 1
    B2 = B.reshape(B.shape[0], -1)
    Bc = B2.mT.contiguous()
    solve_(Lbuf, Bc, nb, **kw)
    X = Bc.mT
    return X.reshape(-1) if vec else X


def factor_solve_batched_(A, a_off, lda, B, b_off, n, nb, nrhs: int, *, policy: int = POLICY_LIST, seed: int = 0,
                          wait_limit_us: int = 0, ws=None, want_kernel_ms: bool = False, trace=None,
                          check: bool = True, wgs=None):
    """Factor and solve many systems in one launch, in place.

    A, B: CUDA float64 1-D tensors holding every system (see
    tchol_factor_solve_batched for the per-system layout given by the host
    arrays a_off, lda, b_off, n and nb).  wgs: optional per-system count of
    workgroups sharing a one-tile system's factorization (tchol_opts.wgs).
    Returns the per-system info array (numpy int32), or (info, kernel_ms)."""
    torch = _torch()
    if A.dtype != torch.float64 or B.dtype != torch.float64 or not A.is_contiguous() or not B.is_contiguous():
        raise ValueError("A and B must be contiguous float64 tensors")
    a_off, b_off, lda, n, nb = _i64(a_off), _i64(b_off), _i32(lda), _i32(n), _i32(nb)
    batch = len(n)
    if not (len(a_off) == len(b_off) == len(lda) == len(nb) == batch):
        raise ValueError("per-system arrays must have the same length")
    if batch and (int(np.max(a_off + lda.astype(np.int64) * n)) > A.numel() or
                  (nrhs and int(np.max(b_off + n.astype(np.int64) * nrhs)) > B.numel())):
        raise ValueError("a system extends past the end of A or B")
    info = np.zeros(max(batch, 1), dtype=np.int32)
    lib = load()
    P32 = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    with torch.cuda.device(A.device):
        need = batched_workspace_bytes(n, nb) if batch else 256
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, A.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace)
        if wgs is not None:
            wgs = _i32(wgs)
            if len(wgs) != batch:
                raise ValueError("wgs must have one entry per system")
            o.wgs = wgs.ctypes.data_as(P32)
        rc = lib.tchol_factor_solve_batched(ctypes.c_void_p(A.data_ptr()), a_off.ctypes.data_as(P64),
                                            lda.ctypes.data_as(P32), ctypes.c_void_p(B.data_ptr()),
                                            b_off.ctypes.data_as(P64), n.ctypes.data_as(P32),
                                            nb.ctypes.data_as(P32), int(nrhs), batch, info.ctypes.data_as(P32),
                                            ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                            _stream_ptr(torch, A.device), ctypes.byref(o))
    if rc != 0 and check:
        raise TcholError(rc, "tchol_factor_solve_batched")
    info = info[:batch]
    return (info, ms.value) if want_kernel_ms else info


def solve_mixed_(A, Bc, nb: int, *, tol: float = 1e-12, maxit: int = 30, lowp: int = LOWP_FP32,
                 policy: int = POLICY_LIST, seed: int = 0, wait_limit_us: int = 0, ws=None,
                 want_kernel_ms: bool = False, trace=None, check: bool = True):
    """Mixed-precision solve with iterative refinement, in place on Bc.

    A: CUDA float64 (n, n) contiguous symmetric (read only).  Bc: CUDA float64
    (nrhs, n) contiguous (B column-major), overwritten by the solution.
    Returns (rc, iters, berr) with berr the final normwise backward error per
    right-hand side (numpy); rc is 0, the failing leading minor of the
    low-precision factorization, or E_NOCONV; with want_kernel_ms a fourth
    entry gives the factorization kernel's time."""
    torch = _torch()
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("A must be a contiguous square float64 tensor")
    n = A.shape[0]
    if Bc.dtype != torch.float64 or not Bc.is_contiguous() or Bc.dim() != 2 or Bc.shape[1] != n:
        raise ValueError("Bc must be a contiguous float64 (nrhs, n) tensor (B in column-major order)")
    nrhs = Bc.shape[0]
    lib = load()
    berr = np.zeros(max(nrhs, 1), dtype=np.float64)
    iters = ctypes.c_int32(0)
    with torch.cuda.device(A.device):
        need = mixed_workspace_bytes(n, nb, nrhs, lowp) if n else 256
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, A.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace)
        rc = lib.tchol_solve_mixed(ctypes.c_void_p(A.data_ptr()), n, nb, ctypes.c_void_p(Bc.data_ptr()), nrhs,
                                   lowp, float(tol), int(maxit), berr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(iters), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_ptr(torch, A.device), ctypes.byref(o))
    if check and rc < 0 and rc != E_NOCONV:
        raise TcholError(rc, "tchol_solve_mixed")
    out = (rc, int(iters.value), berr[:nrhs])
    return out + (ms.value,) if want_kernel_ms else out


def solve_mixed(A, B, nb: int, *, fallback: bool = True, **kw):
    """X = A^{-1} B by the mixed-precision solve; B is (n,) or (n, nrhs).

    When the low-precision factorization breaks down or the refinement does
    not reach tol within maxit, and fallback is set, the system is solved by
    the FP64 path (factor of a copy of A, then the backward-stable solve by
    substitution), as LAPACK's mixed solvers do.  Returns (X, info) with info = {"rc", "iters", "berr",
    "fallback"}."""
    torch = _torch()
    vec = B.dim() == 1
    B2 = B.reshape(B.shape[0], -1)
    Bc = B2.mT.contiguous().to(torch.float64)
    rc, iters, berr = solve_mixed_(A, Bc, nb, **kw)[:3]
    used = False
    if rc != 0 and fallback:
        Lbuf = A.detach().clone()
        info = factor_(Lbuf, nb)
        if info != 0:
            raise TcholError(int(info), "tchol_factor (fallback)")
        Bc = B2.mT.contiguous().to(torch.float64)
        solve_(Lbuf, Bc, nb, subst=True)
        used = True
    elif rc != 0:
        raise TcholError(int(rc), "tchol_solve_mixed")
    X = Bc.mT
    return (X.reshape(-1) if vec else X), {"rc": int(rc), "iters": iters, "berr": berr, "fallback": used}


def backward_(Lbuf, Gb, nb: int, *, policy: int = POLICY_LIST, seed: int = 0, wait_limit_us: int = 0, ws=None,
              want_kernel_ms: bool = False, trace=None, check: bool = True):
    """Adjoint of the factorization, in place.  Lbuf: the (n, n) buffer factored
    by factor_ (column-major lower = L).  Gb: CUDA float64 (n, n) contiguous
    whose column-major lower triangle is Lbar = df/dL (i.e. Gb = Lbar^T in
    row-major terms); on return its column-major lower triangle holds that of
    the symmetric Abar = df/dA.  Returns rc, or (rc, kernel_ms)."""
    torch = _torch()
    n = Lbuf.shape[0]
    for t in (Lbuf, Gb):
        if t.dtype != torch.float64 or t.dim() != 2 or tuple(t.shape) != (n, n) or not t.is_contiguous():
            raise ValueError("L and Lbar must be contiguous float64 (n, n) tensors")
    lib = load()
    with torch.cuda.device(Lbuf.device):
        need = workspace_bytes(OP_BACKWARD, n, nb) if n else 256
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, Lbuf.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace)
        rc = lib.tchol_backward_ex(ctypes.c_void_p(Lbuf.data_ptr()), n, nb, ctypes.c_void_p(Gb.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(torch, Lbuf.device),
                                   ctypes.byref(o))
    if rc != 0 and check:
        raise TcholError(rc, "tchol_backward")
    return (rc, ms.value) if want_kernel_ms else rc


_CHOL_FN = None


def _chol_function():
    global _CHOL_FN
    if _CHOL_FN is not None:
        return _CHOL_FN
    import torch

    class _Cholesky(torch.autograd.Function):
        """L = chol(A) (lower) by the tile factorization; its backward runs the
        library's adjoint and returns the symmetric gradient with respect to A."""

        @staticmethod
        def forward(ctx, A, nb):
            W = A.detach().to(torch.float64).contiguous().clone()
            info = factor_(W, nb)
            if info != 0:
                raise TcholError(int(info), "tchol_factor (matrix not positive definite)")
            ctx.save_for_backward(W)
            ctx.nb = nb
            return torch.tril(W.mT)

        @staticmethod
        def backward(ctx, gL):
            (W,) = ctx.saved_tensors
            Gb = torch.tril(gL.to(torch.float64)).mT.contiguous()   # column-major lower = Lbar
            backward_(W, Gb, ctx.nb)
            low = torch.tril(Gb.mT)
            return low + torch.tril(low, -1).mT, None

    _CHOL_FN = _Cholesky
    return _CHOL_FN


def cholesky(A, nb: int):
    """Differentiable lower Cholesky factor of the symmetric positive definite
    A (CUDA float64; its lower triangle is read).  Gradients flow back to A as
    the symmetric adjoint computed by tchol_backward."""
    _torch()
    return _chol_function().apply(A, nb)


def batched_f32_workspace_bytes(n, nb, nrhs: int) -> int:
    n32, nb32 = _i32(n), _i32(nb)
    P32 = ctypes.POINTER(ctypes.c_int32)
    r = load().tchol_batched_f32_workspace_bytes(n32.ctypes.data_as(P32), nb32.ctypes.data_as(P32), len(n32), nrhs)
    if r < 0:
        raise TcholError(int(r), "tchol_batched_f32_workspace_bytes")
    return int(r)


def factor_solve_batched_f32_(A, a_off, lda, B, b_off, n, nb, nrhs: int, *, policy: int = POLICY_LIST,
                              seed: int = 0, wait_limit_us: int = 0, ws=None, want_kernel_ms: bool = False,
                              trace=None, check: bool = True):
    """Factor and solve many FP32 systems in one launch, in place (FP32 updates,
    FP64 diagonal tiles and solves; see tchol_factor_solve_batched_f32).  A, B:
    CUDA float32 1-D tensors; lda[s] a multiple of 4 and >= n[s] + 3, a_off[s]
    a multiple of 4 (spd_inputs packs them so with align=4, pad=3).  Returns
    the per-system info (numpy int32), or (info, kernel_ms)."""
    torch = _torch()
    if A.dtype != torch.float32 or B.dtype != torch.float32 or not A.is_contiguous() or not B.is_contiguous():
        raise ValueError("A and B must be contiguous float32 tensors")
    a_off, b_off, lda, n, nb = _i64(a_off), _i64(b_off), _i32(lda), _i32(n), _i32(nb)
    batch = len(n)
    if not (len(a_off) == len(b_off) == len(lda) == len(nb) == batch):
        raise ValueError("per-system arrays must have the same length")
    if batch and (int(np.max(a_off + lda.astype(np.int64) * n)) > A.numel() or
                  (nrhs and int(np.max(b_off + n.astype(np.int64) * nrhs)) > B.numel())):
        raise ValueError("a system extends past the end of A or B")
    info = np.zeros(max(batch, 1), dtype=np.int32)
    lib = load()
    P32 = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    with torch.cuda.device(A.device):
        need = batched_f32_workspace_bytes(n, nb, nrhs) if batch else 256
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, A.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace)
        rc = lib.tchol_factor_solve_batched_f32(ctypes.c_void_p(A.data_ptr()), a_off.ctypes.data_as(P64),
                                                lda.ctypes.data_as(P32), ctypes.c_void_p(B.data_ptr()),
                                                b_off.ctypes.data_as(P64), n.ctypes.data_as(P32),
                                                nb.ctypes.data_as(P32), int(nrhs), batch, info.ctypes.data_as(P32),
                                                ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                                _stream_ptr(torch, A.device), ctypes.byref(o))
    if rc != 0 and check:
        raise TcholError(rc, "tchol_factor_solve_batched_f32")
    info = info[:batch]
    return (info, ms.value) if want_kernel_ms else info


def factor_solve_(A, Bc, nb: int, *, policy: int = POLICY_LIST, seed: int = 0, wait_limit_us: int = 0, ws=None,
                  want_kernel_ms: bool = False, trace=None, check: bool = True, subst: bool = False):
    """Factor A in place and solve in place on Bc in one launch (merged DAG).
    A: CUDA float64 (n, n) contiguous symmetric; Bc: CUDA float64 (nrhs, n)
    contiguous (B column-major).  subst: as for solve_.  Returns info (0, or
    the failing leading minor), or (info, kernel_ms)."""
    torch = _torch()
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("A must be a contiguous square float64 tensor")
    n = A.shape[0]
    if Bc.dtype != torch.float64 or not Bc.is_contiguous() or Bc.dim() != 2 or Bc.shape[1] != n:
        raise ValueError("Bc must be a contiguous float64 (nrhs, n) tensor (B in column-major order)")
    nrhs = Bc.shape[0]
    lib = load()
    with torch.cuda.device(A.device):
        need = lib.tchol_factor_solve_workspace_bytes(n, nb, nrhs) if n else 256
        if need < 0:
            raise TcholError(int(need), "tchol_factor_solve_workspace_bytes")
        if ws is None or ws.numel() < need:
            ws = _workspace(torch, need, A.device)
        o, ms = _opts(policy, seed, wait_limit_us, want_kernel_ms, trace, subst)
        rc = lib.tchol_factor_solve(ctypes.c_void_p(A.data_ptr()), n, nb, ctypes.c_void_p(Bc.data_ptr()), nrhs,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(torch, A.device),
                                    ctypes.byref(o))
    if rc < 0 and check:
        raise TcholError(rc, "tchol_factor_solve")
    return (rc, ms.value) if want_kernel_ms else rc


def factor_solve_noalloc_(A, Bc, nb: int, *, check: bool = True):
    """As factor_solve_ (default options, subst=True) through tchol_factor_solve_noalloc:
    the library's fixed per-GPU scratch array instead of a workspace, so
    nothing is allocated on the device by the call.  Returns info."""
    torch = _torch()
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("A must be a contiguous square float64 tensor")
    n = A.shape[0]
    if Bc.dtype != torch.float64 or not Bc.is_contiguous() or Bc.dim() != 2 or Bc.shape[1] != n:
        raise ValueError("Bc must be a contiguous float64 (nrhs, n) tensor (B in column-major order)")
    lib = load()
    with torch.cuda.device(A.device):
        rc = lib.tchol_factor_solve_noalloc(ctypes.c_void_p(A.data_ptr()), n, nb, ctypes.c_void_p(Bc.data_ptr()),
                                            Bc.shape[0], _stream_ptr(torch, A.device))
    if rc < 0 and check:
        raise TcholError(rc, "tchol_factor_solve_noalloc")
    return rc
