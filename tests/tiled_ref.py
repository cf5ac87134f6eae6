"""Test-only tiled Cholesky reference on the CPU (numpy, FP64).

Each tile operation applies its updates one rank-1 term at a time in
ascending order, with every product rounded before it is subtracted, so
every element of the matrix sees exactly the same rounded operations in the
same order as the unblocked right-looking oracle.  Any topological order of
the tile DAG therefore produces the oracle's factor bit for bit.  The tile
tasks are those of the right-looking tile Cholesky (Buttari et al., the
PLASMA algorithm the paper schedules, section 4.1 "Benchmarks"):

    POTRF(k):      A_kk <- chol(A_kk)
    TRSM(i, k):    A_ik <- A_ik L_kk^{-T}                  (i > k)
    SYRK(i, k):    A_ii <- A_ii - L_ik L_ik^T  (lower)     (i > k)
    GEMM(i, j, k): A_ij <- A_ij - L_ik L_jk^T              (i > j > k)
    GEMM2(i, j, k): GEMM(i, j, k), then GEMM(i, j, k + 1)  (two updates of
                    one tile in one task, as the planner merges them)

This module is independent of both the oracle and the GPU library.
"""
from __future__ import annotations

import math
import numpy as np

POTRF, TRSM, SYRK, GEMM = 0, 1, 2, 3
GEMM2 = 14


def tile_bounds(n: int, nb: int, t: int):
    return t * nb, min(n, (t + 1) * nb)


class NotPositiveDefinite(Exception):
    def __init__(self, col):
        super().__init__("pivot %d not positive" % col)
        self.col = col


def tile_potrf(T: np.ndarray, col0: int = 0):
    m = T.shape[0]
    for c in range(m):
        d = T[c, c]
        if not (d > 0.0):
            raise NotPositiveDefinite(col0 + c + 1)
        T[c, c] = math.sqrt(d)
        T[c + 1:, c] = T[c + 1:, c] / T[c, c]
        for j in range(c + 1, m):
            T[j:, j] = T[j:, j] - T[j:, c] * T[j, c]


def tile_trsm(X: np.ndarray, Lkk: np.ndarray):
    m = Lkk.shape[0]
    for c in range(m):
        X[:, c] = X[:, c] / Lkk[c, c]
        for c2 in range(c + 1, m):
            X[:, c2] = X[:, c2] - X[:, c] * Lkk[c2, c]


def tile_syrk(C: np.ndarray, X: np.ndarray):
    mi, mk = X.shape
    for q in range(mk):
        for j in range(mi):
            C[j:, j] = C[j:, j] - X[j:, q] * X[j, q]


def tile_gemm(C: np.ndarray, X: np.ndarray, Y: np.ndarray):
    for q in range(X.shape[1]):
        C[:, :] = C - np.multiply.outer(X[:, q], Y[:, q])


def run_task(A: np.ndarray, n: int, nb: int, kind: int, i: int, j: int, k: int):
    """Apply one tile task in place to the (row-major numpy) matrix A."""
    ri0, ri1 = tile_bounds(n, nb, i)
    rj0, rj1 = tile_bounds(n, nb, j)
    rk0, rk1 = tile_bounds(n, nb, k)
    if kind == POTRF:
        tile_potrf(A[rk0:rk1, rk0:rk1], rk0)
    elif kind == TRSM:
        tile_trsm(A[ri0:ri1, rk0:rk1], A[rk0:rk1, rk0:rk1])
    elif kind == SYRK:
        tile_syrk(A[ri0:ri1, ri0:ri1], A[ri0:ri1, rk0:rk1])
    elif kind == GEMM:
        tile_gemm(A[ri0:ri1, rj0:rj1], A[ri0:ri1, rk0:rk1], A[rj0:rj1, rk0:rk1])
    elif kind == GEMM2:
        rl0, rl1 = tile_bounds(n, nb, k + 1)
        tile_gemm(A[ri0:ri1, rj0:rj1], A[ri0:ri1, rk0:rk1], A[rj0:rj1, rk0:rk1])
        tile_gemm(A[ri0:ri1, rj0:rj1], A[ri0:ri1, rl0:rl1], A[rj0:rj1, rl0:rl1])
    else:
        raise ValueError(kind)


TRTRI = 12


def pair_first(j: int, k: int) -> bool:
    """Update k of a tile in column j opens a merged pair (k, k + 1): k even,
    and the pair does not hold the tile's last update j - 1."""
    return k % 2 == 0 and k + 1 <= j - 2


def pair_second(j: int, k: int) -> bool:
    return k % 2 == 1 and k <= j - 2


def factor_program(T: int, tri: bool = False):
    """The factorization's tasks in program order (k outer), with each merged
    pair of updates placed at its second step, and every task's tile reads and
    writes: [(task, reads, writes)].  With ``tri`` (the merged factor + solve
    launch), TRSM(i, k) applies the inverse ("D", k) that TRTRI(k) makes from
    L_kk after POTRF(k), for k < T - 1."""
    out = []
    for k in range(T):
        out.append(((POTRF, k, k, k), [(k, k)], [(k, k)]))
        if tri and k + 1 < T:
            out.append(((TRTRI, k, k, k), [(k, k)], [("D", k)]))
        for i in range(k + 1, T):
            out.append(((TRSM, i, k, k), [("D", k) if tri else (k, k), (i, k)], [(i, k)]))
        for i in range(k + 1, T):
            out.append(((SYRK, i, i, k), [(i, k), (i, i)], [(i, i)]))
            for j in range(k + 1, i):
                if pair_first(j, k):
                    continue
                if pair_second(j, k):
                    out.append(((GEMM2, i, j, k - 1), [(i, k - 1), (j, k - 1), (i, k), (j, k), (i, j)], [(i, j)]))
                else:
                    out.append(((GEMM, i, j, k), [(i, k), (j, k), (i, j)], [(i, j)]))
    return out


FTRSV, FGEMV, BTRSV, BGEMV = 4, 5, 6, 7


def solve_program(T: int, inv=(), given=()):
    """The forward then backward tiled substitution's tasks in program order,
    with the data each reads and writes: tiles ("L", i, j) of the factor,
    blocks ("B", i) of the right-hand sides, and, for the diagonal tiles k in
    ``inv`` (the FP64 solve's explicit inverses), the inverse ("D", k) made by
    TRTRI(k) and the intermediate block ("S", k) that holds y_k.  A diagonal
    step of a tile not in ``inv`` substitutes in place in B.  The inverses of
    the tiles in ``given`` were made by the factorization's own TRTRI tasks."""
    inv = set(inv)
    given = set(given)
    y = lambda k: ("S", k) if k in inv else ("B", k)  # where y_k lives
    out = []
    for k in range(T):
        if k in inv:
            if k not in given:
                out.append(((TRTRI, k, k, k), [("L", k, k)], [("D", k)]))
            out.append(((FTRSV, k, k, k), [("D", k), ("B", k)], [("S", k)]))
        else:
            out.append(((FTRSV, k, k, k), [("L", k, k), ("B", k)], [("B", k)]))
        for i in range(k + 1, T):
            out.append(((FGEMV, i, k, k), [("L", i, k), y(k), ("B", i)], [("B", i)]))
    for k in range(T - 1, -1, -1):
        if k in inv:
            out.append(((BTRSV, k, k, k), [("D", k), ("S", k)], [("B", k)]))
        else:
            out.append(((BTRSV, k, k, k), [("L", k, k), ("B", k)], [("B", k)]))
        for i in range(k):
            out.append(((BGEMV, i, k, k), [("L", k, i), ("B", k), y(i)], [y(i)]))
    return out


def tasks_k_major(n: int, nb: int):
    """Tile tasks in the textbook loop order (k outer)."""
    T = (n + nb - 1) // nb
    out = []
    for k in range(T):
        out.append((POTRF, k, k, k))
        for i in range(k + 1, T):
            out.append((TRSM, i, k, k))
        for i in range(k + 1, T):
            out.append((SYRK, i, i, k))
            for j in range(k + 1, i):
                out.append((GEMM, i, j, k))
    return out


def tiled_cholesky(A: np.ndarray, nb: int, order=None):
    """Factor a copy of A with the tile algorithm; returns (L_lower_full_array, info)."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    order = tasks_k_major(n, nb) if order is None else order
    try:
        for kind, i, j, k in order:
            run_task(A, n, nb, kind, i, j, k)
    except NotPositiveDefinite as e:
        return A, e.col
    return A, 0
