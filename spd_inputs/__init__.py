"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no Cholesky arithmetic: it only draws random numbers and
forms the symmetric positive definite test matrices.  The paper measures on
FP64 matrices of order 8192 and 16384 tiled by 512 (section 4, "Methodology"
and "Impact of the affinity control parameter") but never says how they were
generated; the family used here stands in for them:

    rng = numpy.random.default_rng(seed)          # PCG64
    B   = rng.uniform(-1, 1, (n, n))              # float64, row-major draw order
    A   = (B @ B.T) / n + shift * I               # made exactly symmetric
    rhs = rng.uniform(-1, 1, (n, nrhs))           # drawn next from the same stream

``shift`` is 1 for the plain FP64 workloads (condition number about 2.3) and
1e-4 for the mixed-precision workload (condition number about 1.3e4).

Batched workloads draw the orders first, ``ns = rng.integers(lo, hi + 1,
count)``, then, system by system in index order, B_i (n_i x n_i) and the
right-hand sides b_i (n_i x nrhs) from the same stream, with
A_i = B_i B_i^T / n_i + shift I.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "spd_matrix", "spd_matrix_and_rhs", "draw_uniform_rows", "rhs", "integer_factor",
    "integer_spd", "integer_rhs", "lower_upstream", "batched_sizes", "batched_systems", "pack_batched",
    "batched_systems_device",
]


def draw_uniform_rows(rng: np.random.Generator, n: int, cols: int, chunk_rows: int = 2048):
    """Yield (row0, block) pieces of rng.uniform(-1, 1, (n, cols)) in draw order.

    Drawing the rows in chunks consumes the generator exactly as one call for
    the whole (n, cols) array would, so large matrices can be streamed.
    """
    r = 0
    while r < n:
        m = min(chunk_rows, n - r)
        yield r, rng.uniform(-1.0, 1.0, (m, cols))
        r += m


def spd_matrix(n: int, seed: int, shift: float = 1.0):
    """Return (A, rng): A = B B^T / n + shift I (exactly symmetric, float64 C-order)."""
    rng = np.random.default_rng(seed)
    B = rng.uniform(-1.0, 1.0, (n, n))
    A = (B @ B.T) / float(max(n, 1))
    A = np.tril(A) + np.tril(A, -1).T
    A[np.diag_indices(n)] += shift
    return A, rng


def rhs(rng: np.random.Generator, n: int, nrhs: int) -> np.ndarray:
    """Right-hand sides U[-1, 1], (n, nrhs), drawn next from ``rng``."""
    return rng.uniform(-1.0, 1.0, (n, nrhs))


def spd_matrix_and_rhs(n: int, seed: int, nrhs: int, shift: float = 1.0):
    A, rng = spd_matrix(n, seed, shift)
    return A, rhs(rng, n, nrhs)


def integer_factor(n: int, seed: int) -> np.ndarray:
    """Lower-triangular L0 with diagonal in {1, 2, 4} and off-diagonal in {-2..2}.

    Powers of two on the diagonal make sqrt, division and reciprocal
    multiplication exact, and A = L0 L0^T has small integer entries, so an
    exact Cholesky implementation must return L0 bit for bit.
    """
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-2, 3, (n, n)).astype(np.float64), -1)
    L[np.diag_indices(n)] = rng.choice(np.array([1.0, 2.0, 4.0]), n)
    return L


def integer_spd(n: int, seed: int):
    """Return (A, L0) with A = L0 L0^T computed exactly (integers below 2^53)."""
    L0 = integer_factor(n, seed)
    Li = L0.astype(np.int64)
    A = (Li @ Li.T).astype(np.float64)
    return A, L0


def integer_rhs(A: np.ndarray, nrhs: int, seed: int):
    """Return (b, x0): integer x0 in {-3..3} and b = A x0 computed exactly."""
    rng = np.random.default_rng(seed + 1000003)
    x0 = rng.integers(-3, 4, (A.shape[0], nrhs)).astype(np.int64)
    b = (A.astype(np.int64) @ x0).astype(np.float64)
    return b, x0.astype(np.float64)


def lower_upstream(rng: np.random.Generator, n: int) -> np.ndarray:
    """Upstream gradient Lbar: lower-triangular with N(0, 1) entries, drawn next from ``rng``."""
    return np.tril(rng.standard_normal((n, n)))


def batched_sizes(count: int, seed: int, lo: int = 16, hi: int = 512):
    """Sizes n_i uniform on the integers [lo, hi] and the generator to draw the systems from."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count), rng


def spd_matrix_device(n: int, seed: int, shift: float = 1.0, device="cuda", chunk_rows: int = 2048):
    """The same recipe as :func:`spd_matrix` for orders too large for a host GEMM.

    B is drawn on the host from the same PCG64 stream, in row chunks, and
    copied to the device; A = B B^T / n is formed there with torch's FP64
    matrix product (input generation only), made exactly symmetric from its
    lower triangle, and shifted.  The product's rounding differs from the
    host version, so exact comparisons use the device A itself.  Returns
    (A, rng) with A a contiguous (n, n) float64 tensor on ``device``.
    """
    import torch

    rng = np.random.default_rng(seed)
    B = torch.empty((n, n), dtype=torch.float64, device=device)
    for r0, blk in draw_uniform_rows(rng, n, n, chunk_rows):
        B[r0:r0 + blk.shape[0]].copy_(torch.from_numpy(blk))
    Bt = B.t().contiguous()
    A = torch.matmul(B, Bt)
    del Bt, B
    A.div_(float(max(n, 1)))
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        # upper part of these rows := transpose of the lower part of these columns
        A[r0:r1, r1:] = A[r1:, r0:r1].t()
        blk = A[r0:r1, r0:r1]
        blk.copy_(torch.tril(blk) + torch.tril(blk, -1).t())
    A.diagonal().add_(shift)
    return A, rng


def _sym_from_lower(A: np.ndarray) -> np.ndarray:
    return np.tril(A) + np.tril(A, -1).T


def batched_systems(count: int, seed: int, nrhs: int, shift: float = 1.0, lo: int = 16, hi: int = 512,
                    sizes=None):
    """Host recipe of a batch: returns (ns, [A_i], [b_i]).  With ``sizes``
    given, the orders are not drawn (the stream starts with B_0)."""
    rng = np.random.default_rng(seed)
    ns = np.asarray(sizes, dtype=np.int64) if sizes is not None else rng.integers(lo, hi + 1, size=count)
    As, bs = [], []
    for n in ns:
        n = int(n)
        B = rng.uniform(-1.0, 1.0, (n, n))
        A = _sym_from_lower((B @ B.T) / float(max(n, 1)))
        A[np.diag_indices(n)] += shift
        As.append(A)
        bs.append(rng.uniform(-1.0, 1.0, (n, nrhs)))
    return ns, As, bs


def _layout(ns, nrhs: int, align: int, pad: int = 0):
    """Column-major packing: lda_i = n_i + pad rounded up to ``align`` (>= 1),
    every A_i starting at a multiple of ``align`` elements; B_i packed with
    ld n_i.  (The FP32 batched launch takes align = 4, pad = 3.)"""
    ns = np.asarray(ns, dtype=np.int64)
    lda = np.maximum(1, (ns + pad + align - 1) // align * align)
    sizes_a = lda * ns
    a_off = np.concatenate([[0], np.cumsum(sizes_a)[:-1]]) if len(ns) else np.zeros(0, np.int64)
    b_off = np.concatenate([[0], np.cumsum(ns * nrhs)[:-1]]) if len(ns) else np.zeros(0, np.int64)
    return lda.astype(np.int64), a_off.astype(np.int64), b_off.astype(np.int64), int(sizes_a.sum()), \
        int((ns * nrhs).sum())


def pack_batched(As, bs, align: int = 2, pad: int = 0, dtype=np.float64):
    """Pack host systems into flat column-major arrays of ``dtype``.  Returns
    (A_flat, a_off, lda, B_flat, b_off) as numpy arrays."""
    ns = [a.shape[0] for a in As]
    nrhs = bs[0].shape[1] if bs else 0
    lda, a_off, b_off, na, nbt = _layout(ns, nrhs, align, pad)
    Af = np.zeros(max(na, 1), dtype=dtype)
    Bf = np.zeros(max(nbt, 1), dtype=dtype)
    for A, b, o, l, ob in zip(As, bs, a_off, lda, b_off):
        n = A.shape[0]
        # column c of A (column-major) is row c of the symmetric A
        Af[o:o + n * l].reshape(n, l)[:, :n] = A
        Bf[ob:ob + n * nrhs].reshape(nrhs, n)[:] = b.T
    return Af, a_off, lda, Bf, b_off


def batched_systems_device(count: int, seed: int, nrhs: int, shift: float = 1.0, lo: int = 16, hi: int = 512,
                           align: int = 2, device="cuda", sizes=None, pad: int = 0, fp32: bool = False):
    """The batched recipe with the products formed on the device (input
    generation only, in FP64), packed as :func:`pack_batched` does (rounded to
    FP32 with ``fp32``).  Returns (ns, A_flat, a_off, lda, B_flat, b_off) with
    A_flat, B_flat device tensors."""
    import torch

    rng = np.random.default_rng(seed)
    ns = np.asarray(sizes, dtype=np.int64) if sizes is not None else rng.integers(lo, hi + 1, size=count)
    lda, a_off, b_off, na, nbt = _layout(ns, nrhs, align, pad)
    dt = torch.float32 if fp32 else torch.float64
    Af = torch.zeros(max(na, 1), dtype=dt, device=device)
    Bf = torch.zeros(max(nbt, 1), dtype=dt, device=device)
    for n, o, l, ob in zip(ns, a_off, lda, b_off):
        n, o, l, ob = int(n), int(o), int(l), int(ob)
        B = torch.from_numpy(rng.uniform(-1.0, 1.0, (n, n))).to(device)
        A = torch.matmul(B, B.t().contiguous()) / float(max(n, 1))
        A = torch.tril(A) + torch.tril(A, -1).t()
        A.diagonal().add_(shift)
        Af[o:o + n * l].view(n, l)[:, :n].copy_(A)
        b = torch.from_numpy(rng.uniform(-1.0, 1.0, (n, nrhs))).to(device)
        Bf[ob:ob + n * nrhs].view(nrhs, n).copy_(b.t())
    return ns, Af, a_off, lda, Bf, b_off
