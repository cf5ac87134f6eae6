"""Pins of the CPU oracle against facts the mathematics fixes.

The paper prints no worked example or numbers for its Cholesky workload, so
the oracle is pinned by: exact recovery of a known integer factor; the
backward-error bound of Cholesky (Higham, Accuracy and Stability of Numerical
Algorithms, ch. 10); agreement with LAPACK's dpotrf; bitwise equality with an
independent tiled reference; special cases with closed forms; and a mutation
test showing that plausible slips in the oracle source break these pins.
"""
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg

import spd_inputs
from tests import tiled_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return rows


def test_textbook_3x3(oracle_lib):
    rows = _read_golden("textbook_3x3.txt")
    A, L = np.array(rows[0:3]), np.array(rows[3:6])
    b, x = np.array(rows[6]), np.array(rows[7])
    F, info = oracle_lib.potrf(A)
    assert info == 0
    assert np.array_equal(np.tril(F), L)
    assert np.array_equal(oracle_lib.potrs(F, b), x)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 255])
def test_exact_integer_recovery(oracle_lib, n):
    A, L0 = spd_inputs.integer_spd(n, seed=n)
    F, info = oracle_lib.potrf(A)
    assert info == 0
    assert np.array_equal(np.tril(F), L0)
    b, x0 = spd_inputs.integer_rhs(A, 3, seed=n)
    assert np.array_equal(oracle_lib.potrs(F, b), x0)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 255, 1024])
def test_backward_error_bound(oracle_lib, n):
    A, _ = spd_inputs.spd_matrix(n, seed=n, shift=1.0)
    F, info = oracle_lib.potrf(A)
    assert info == 0
    assert oracle_lib.backward_error(A, F) <= 10.0


@pytest.mark.parametrize("n,shift", [(512, 1.0), (1024, 1.0), (768, 1e-4)])
def test_matches_lapack(oracle_lib, n, shift):
    A, _ = spd_inputs.spd_matrix(n, seed=7, shift=shift)
    F, info = oracle_lib.potrf(A)
    assert info == 0
    L_lapack = scipy.linalg.cholesky(A, lower=True)
    tol = 1e-13 if shift == 1.0 else 1e-9  # forward error scales with cond(A)
    assert oracle_lib.factor_error(F, L_lapack) <= tol


def test_upper_triangle_ignored_and_untouched(oracle_lib):
    A, _ = spd_inputs.spd_matrix(40, seed=3)
    G = np.array(A)
    G[np.triu_indices(40, 1)] = np.nan
    F1, i1 = oracle_lib.potrf(A)
    F2, i2 = oracle_lib.potrf(G)
    assert i1 == i2 == 0
    assert np.array_equal(np.tril(F1), np.tril(F2))
    assert np.all(np.isnan(F2[np.triu_indices(40, 1)]))
    assert np.array_equal(F1[np.triu_indices(40, 1)], A[np.triu_indices(40, 1)])


def test_special_cases(oracle_lib):
    F, info = oracle_lib.potrf(np.zeros((0, 0)))
    assert info == 0 and F.shape == (0, 0)
    F, info = oracle_lib.potrf(np.array([[2.25]]))
    assert info == 0 and F[0, 0] == 1.5
    d = np.array([4.0, 9.0, 0.25, 2.0])
    F, info = oracle_lib.potrf(np.diag(d))
    assert info == 0 and np.array_equal(np.diag(F), np.sqrt(d))
    assert np.array_equal(np.tril(F, -1), np.zeros((4, 4)))


@pytest.mark.parametrize("j", [0, 5, 29])
@pytest.mark.parametrize("how", ["zero", "negative", "nan"])
def test_breakdown_info(oracle_lib, j, how):
    A, L0 = spd_inputs.integer_spd(30, seed=11)
    if how == "zero":
        A[j, j] -= L0[j, j] ** 2          # pivot of column j becomes exactly 0
    elif how == "negative":
        A[j, j] -= L0[j, j] ** 2 + 1.0    # pivot becomes exactly -1
    else:
        A[j, j] = np.nan
    F, info = oracle_lib.potrf(A)
    assert info == j + 1
    # the columns before the failing one are already final
    assert np.array_equal(np.tril(F)[:, :j], L0[:, :j])


def test_solve_accuracy_and_lapack(oracle_lib):
    A, B = spd_inputs.spd_matrix_and_rhs(300, seed=5, nrhs=4)
    L = oracle_lib.cholesky(A)
    X = oracle_lib.potrs(L, B)
    eta = oracle_lib.solve_backward_error(A, X, B)
    assert np.all(eta <= 1e-15)
    Xs = scipy.linalg.cho_solve((L, True), B)
    assert np.max(np.abs(X - Xs)) / np.max(np.abs(Xs)) <= 1e-13


def test_residual_and_llt_entry_helpers(oracle_lib):
    A, _ = spd_inputs.integer_spd(20, seed=2)
    b, x0 = spd_inputs.integer_rhs(A, 2, seed=2)
    assert np.array_equal(oracle_lib.residual(A, x0, b), np.zeros_like(b))
    L0 = spd_inputs.integer_factor(20, seed=2)
    Lf = np.asfortranarray(L0)
    for (i, j) in [(0, 0), (19, 3), (7, 7), (4, 12)]:
        assert oracle_lib.llt_entry(Lf, i, j) == A[i, j]


@pytest.mark.parametrize("n,nb", [(1, 8), (13, 8), (45, 16), (64, 16), (96, 32), (96, 8)])
def test_tiled_reference_bitwise_equals_oracle(oracle_lib, n, nb):
    A, _ = spd_inputs.spd_matrix(n, seed=n + nb)
    F, info = oracle_lib.potrf(A)
    T, tinfo = tiled_ref.tiled_cholesky(A, nb)
    assert info == tinfo == 0
    assert np.array_equal(np.tril(F), np.tril(T))


def test_tiled_reference_breakdown_matches(oracle_lib):
    A, L0 = spd_inputs.integer_spd(40, seed=4)
    A[21, 21] -= L0[21, 21] ** 2
    _, info = oracle_lib.potrf(A)
    _, tinfo = tiled_ref.tiled_cholesky(A, 8)
    assert info == tinfo == 22


def test_chunked_generator_matches_whole_draw():
    rng1 = np.random.default_rng(9)
    whole = rng1.uniform(-1, 1, (50, 30))
    rng2 = np.random.default_rng(9)
    parts = np.vstack([blk for _, blk in spd_inputs.draw_uniform_rows(rng2, 50, 30, chunk_rows=7)])
    assert np.array_equal(whole, parts)


# ------------------------------------------------------------------ mutation test
# Each entry plants one plausible slip in a private copy of the oracle source;
# the pins above must notice every one of them.
MUTANTS = {
    "sign_of_update": ("AT(A, lda, i, j) - AT(A, lda, i, k) * l_jk", "AT(A, lda, i, j) + AT(A, lda, i, k) * l_jk"),
    "transposed_operand": ("AT(A, lda, i, j) - AT(A, lda, i, k) * l_jk", "AT(A, lda, i, j) - AT(A, lda, k, i) * l_jk"),
    "dropped_division": ("AT(A, lda, i, k) = AT(A, lda, i, k) / l_kk;", "AT(A, lda, i, k) = AT(A, lda, i, k);"),
    "wrong_loop_start": ("for (int64_t i = j; i < n; ++i)", "for (int64_t i = j + 1; i < n; ++i)"),
    "forward_sub_index": ("s = s - AT(L, ldl, i, k) * b[k];", "s = s - AT(L, ldl, k, i) * b[k];"),
}


def _pins_pass(lib_path):
    import ctypes
    lib = ctypes.CDLL(lib_path)
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_potrf.restype = i64
    lib.oracle_potrf.argtypes = [i64, vp, i64]
    lib.oracle_potrs.argtypes = [i64, vp, i64, i64, vp, i64]
    A, L0 = spd_inputs.integer_spd(24, seed=24)
    F = np.asfortranarray(A.copy())
    G = np.array(F, order="F")
    G[np.triu_indices(24, 1)] = np.nan
    info = lib.oracle_potrf(24, G.ctypes.data_as(vp), 24)
    if info != 0 or not np.array_equal(np.tril(G), L0):
        return False
    b, x0 = spd_inputs.integer_rhs(A, 1, seed=24)
    bf = np.asfortranarray(b.copy())
    lib.oracle_potrs(24, np.asfortranarray(L0).ctypes.data_as(vp), 24, 1, bf.ctypes.data_as(vp), 24)
    return np.array_equal(bf, x0)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(oracle_lib, name):
    src = open(os.path.join(os.path.dirname(oracle_lib.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, "mutation anchor vanished from oracle.c: %s" % name
    tmp = tempfile.mkdtemp()
    try:
        csrc = os.path.join(tmp, "m.c")
        so = os.path.join(tmp, "m.so")
        with open(csrc, "w") as f:
            f.write(src.replace(old, new, 1))
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", csrc, "-o", so, "-lm"], check=True)
        assert not _pins_pass(so)
        # and the unmutated source passes the same check
        csrc2 = os.path.join(tmp, "ok.c")
        so2 = os.path.join(tmp, "ok.so")
        with open(csrc2, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", csrc2, "-o", so2, "-lm"], check=True)
        assert _pins_pass(so2)
    finally:
        shutil.rmtree(tmp)
