"""CPU oracle for the tiled Cholesky path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never includes, links, loads or calls it, and it never imports the GPU
library: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, contraction off, OpenMP
over independent columns).  This module only builds that file, marshals numpy
arrays into column-major buffers, and computes the error measures the tests
use.  The paper names the computation (PLASMA's tile DPOTRF in double
precision, section 4.1 "Benchmarks" and "Methodology") but prints no code and
no numbers for it, so the oracle follows the textbook definition of the
Cholesky factor and of forward/back substitution.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EPS = 2.0 ** -52  # unit roundoff convention for FP64 used by the error measures


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, dp, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    lib.oracle_potrf.restype = i64
    lib.oracle_potrf.argtypes = [i64, vp, i64]
    lib.oracle_potrs.restype = None
    lib.oracle_potrs.argtypes = [i64, vp, i64, i64, vp, i64]
    lib.oracle_residual.restype = None
    lib.oracle_residual.argtypes = [i64, vp, i64, i64, vp, i64, vp, i64, vp, i64]
    lib.oracle_chol_adjoint.restype = None
    lib.oracle_chol_adjoint.argtypes = [i64, vp, i64, vp, i64]
    lib.oracle_llt_entry.restype = ctypes.c_double
    lib.oracle_llt_entry.argtypes = [vp, i64, i64, i64]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    del dp
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def potrf(A: np.ndarray):
    """Cholesky factor of the symmetric matrix whose lower triangle is ``A``.

    Returns ``(L, info)``: ``L`` is a new Fortran-ordered array whose lower
    triangle is the factor (strict upper triangle copied unchanged from
    ``A``), ``info`` is 0 or the 1-based column of the first pivot that is not
    positive (LAPACK's convention).  ``A`` itself is not modified.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    F = np.array(A, dtype=np.float64, order="F", copy=True)
    info = _load().oracle_potrf(n, _ptr(F), max(n, 1))
    return F, int(info)


def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower factor L (strict upper triangle zeroed); raises on breakdown."""
    F, info = potrf(A)
    if info != 0:
        raise np.linalg.LinAlgError("matrix not positive definite (info=%d)" % info)
    return np.tril(F)


def potrs(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve (L L^T) X = B by forward then back substitution; returns X."""
    L = np.asarray(L, dtype=np.float64)
    n = L.shape[0]
    Lf = np.array(L, dtype=np.float64, order="F", copy=True)
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    Bf = np.array(B.reshape(n, -1), dtype=np.float64, order="F", copy=True)
    _load().oracle_potrs(n, _ptr(Lf), max(n, 1), Bf.shape[1], _ptr(Bf), max(n, 1))
    return Bf[:, 0].copy() if vec else Bf


def residual(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """R = B - A X (A symmetric, read from its lower triangle), accumulated in long double."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Af = np.asfortranarray(A)
    vec = np.asarray(X).ndim == 1
    Xf = np.array(np.asarray(X, dtype=np.float64).reshape(n, -1), order="F", copy=True)
    Bf = np.array(np.asarray(B, dtype=np.float64).reshape(n, -1), order="F", copy=True)
    Rf = np.zeros_like(Xf, order="F")
    _load().oracle_residual(n, _ptr(Af), max(n, 1), Xf.shape[1], _ptr(Xf), max(n, 1), _ptr(Bf), max(n, 1),
                            _ptr(Rf), max(n, 1))
    return Rf[:, 0].copy() if vec else Rf


def chol_adjoint(L: np.ndarray, Lbar: np.ndarray) -> np.ndarray:
    """Abar = df/dA (symmetric, returned in full) for the Cholesky factor L of
    A and the upstream Lbar = df/dL (lower triangles used), by the reverse of
    the oracle's own factorization steps (see oracle_chol_adjoint)."""
    L = np.asarray(L, dtype=np.float64)
    n = L.shape[0]
    Lf = np.array(np.tril(L), dtype=np.float64, order="F", copy=True)
    Pf = np.array(np.tril(np.asarray(Lbar, dtype=np.float64)), order="F", copy=True)
    _load().oracle_chol_adjoint(n, _ptr(Lf), max(n, 1), _ptr(Pf), max(n, 1))
    low = np.tril(Pf)
    return low + np.tril(low, -1).T


def llt_entry(L: np.ndarray, i: int, j: int) -> float:
    """(L L^T)_ij in long double, for a Fortran-ordered lower factor L."""
    Lf = L if (L.flags.f_contiguous and L.dtype == np.float64) else np.asfortranarray(L, dtype=np.float64)
    return float(_load().oracle_llt_entry(_ptr(Lf), Lf.shape[0], int(i), int(j)))


# ---------------------------------------------------------------- error measures

def sym_from_lower(A: np.ndarray) -> np.ndarray:
    """Symmetric matrix defined by the lower triangle of A."""
    A = np.asarray(A, dtype=np.float64)
    return np.tril(A) + np.tril(A, -1).T


def backward_error(A: np.ndarray, L: np.ndarray) -> float:
    """Scaled backward error ||A - L L^T||_F / (n * eps * ||A||_F) (Higham, ch. 10)."""
    S = sym_from_lower(A)
    Lt = np.tril(np.asarray(L, dtype=np.float64))
    n = S.shape[0]
    if n == 0:
        return 0.0
    E = S - Lt @ Lt.T
    return float(np.linalg.norm(E) / (n * EPS * np.linalg.norm(S)))


def factor_error(L_hat: np.ndarray, L_ref: np.ndarray) -> float:
    """Normwise-max entry error max|L_hat - L| / max|L| over the lower triangle."""
    a = np.tril(np.asarray(L_hat, dtype=np.float64))
    b = np.tril(np.asarray(L_ref, dtype=np.float64))
    den = float(np.max(np.abs(b))) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a - b))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


def solve_backward_error(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Normwise backward error per right-hand side (Rigal and Gaches):
    eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), residual in long double."""
    S = sym_from_lower(A)
    n = S.shape[0]
    X2 = np.asarray(X, dtype=np.float64).reshape(n, -1)
    B2 = np.asarray(B, dtype=np.float64).reshape(n, -1)
    R = residual(A, X2, B2)
    anorm = float(np.max(np.sum(np.abs(S), axis=1))) if n else 0.0
    den = anorm * np.max(np.abs(X2), axis=0) + np.max(np.abs(B2), axis=0)
    return np.max(np.abs(R), axis=0) / den


def relative_residual(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """||b - A x||_inf / ||b||_inf per right-hand side, residual in long double."""
    n = np.asarray(A).shape[0]
    X2 = np.asarray(X, dtype=np.float64).reshape(n, -1)
    B2 = np.asarray(B, dtype=np.float64).reshape(n, -1)
    R = residual(A, X2, B2)
    return np.max(np.abs(R), axis=0) / np.max(np.abs(B2), axis=0)
