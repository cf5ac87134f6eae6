"""Pins of the oracle's Cholesky adjoint against facts that do not depend on
its code (no GPU).

f(A) = <Lbar, chol(A)> has the derivative Abar (symmetric); each check below
comes from a different route:
  - the closed form Abar = sym(L^{-T} Phi(L^T Lbar) L^{-1}), Phi = lower
    triangle with the diagonal halved, evaluated with LAPACK triangular
    solves (a different algorithm from the oracle's reverse sweep);
  - central finite differences of the oracle's forward factorization,
    h = 1e-6: (f(A + hS) - f(A - hS)) / 2h equals 2 Abar_ij for
    S = E_ij + E_ji and Abar_ii for S = E_ii, to 1e-6 of max |Abar|;
  - log det A = 2 sum log L_ii, whose derivative is A^{-1}: with
    Lbar = diag(2 / L_ii) the adjoint must equal numpy's inverse;
  - n = 1 in closed form (a = l^2: Abar = lbar / (2 l)), zero in zero out,
    and linearity in Lbar.
A dropped term, a missing factor 2 or 1/2, or a transposed operand in the
reverse sweep fails the closed form and the finite differences.
"""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle
import spd_inputs


def closed_form(L, Lbar):
    L = np.tril(L)
    M = np.tril(L.T @ np.tril(Lbar))
    M[np.diag_indices_from(M)] *= 0.5
    X = solve_triangular(L, M, trans="T", lower=True)           # L^{-T} M
    G = solve_triangular(L, X.T, trans="T", lower=True).T       # X L^{-1}
    return 0.5 * (G + G.T)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (17, 3), (64, 4), (200, 5)])
def test_adjoint_matches_closed_form(n, seed):
    A, rng = spd_inputs.spd_matrix(n, seed)
    L = oracle.cholesky(A)
    Lbar = spd_inputs.lower_upstream(rng, n)
    got = oracle.chol_adjoint(L, Lbar)
    ref = closed_form(L, Lbar)
    assert np.allclose(got, got.T, rtol=0, atol=0)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_adjoint_matches_central_differences_n48():
    n, h = 48, 1e-6
    A, rng = spd_inputs.spd_matrix(n, 3)
    Lbar = spd_inputs.lower_upstream(rng, n)
    got = oracle.chol_adjoint(oracle.cholesky(A), Lbar)

    def f(M):
        return float(np.sum(np.tril(Lbar) * oracle.cholesky(M)))

    scale = np.max(np.abs(got))
    rs = np.random.default_rng(0)
    pairs = [(i, i) for i in range(0, n, 7)] + [tuple(sorted(rs.integers(0, n, 2), reverse=True)) for _ in range(40)]
    for i, j in pairs:
        S = np.zeros((n, n))
        S[i, j] += 1.0
        if i != j:
            S[j, i] += 1.0
        fd = (f(A + h * S) - f(A - h * S)) / (2 * h)
        want = got[i, j] if i == j else 2.0 * got[i, j]
        assert abs(fd - want) <= 1e-6 * scale, (i, j, fd, want)


@pytest.mark.parametrize("n,shift", [(100, 1.0), (257, 1e-2)])
def test_logdet_gradient_is_inverse(n, shift):
    A, _ = spd_inputs.spd_matrix(n, 7, shift=shift)
    L = oracle.cholesky(A)
    got = oracle.chol_adjoint(L, np.diag(2.0 / np.diag(L)))
    inv = np.linalg.inv(A)
    assert np.max(np.abs(got - inv)) / np.max(np.abs(inv)) <= 1e-10


def test_order_one_zero_and_linearity():
    got = oracle.chol_adjoint(np.array([[3.0]]), np.array([[1.5]]))
    assert got[0, 0] == 1.5 / 6.0
    A, rng = spd_inputs.spd_matrix(30, 9)
    L = oracle.cholesky(A)
    assert np.all(oracle.chol_adjoint(L, np.zeros((30, 30))) == 0.0)
    b1, b2 = spd_inputs.lower_upstream(rng, 30), spd_inputs.lower_upstream(rng, 30)
    lhs = oracle.chol_adjoint(L, 2.0 * b1 - 0.5 * b2)
    rhs = 2.0 * oracle.chol_adjoint(L, b1) - 0.5 * oracle.chol_adjoint(L, b2)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(lhs))


def test_upper_triangle_of_inputs_ignored():
    A, rng = spd_inputs.spd_matrix(20, 11)
    L = oracle.cholesky(A)
    Lbar = spd_inputs.lower_upstream(rng, 20)
    noisy_L = L + np.triu(np.full((20, 20), np.nan), 1)
    noisy_b = Lbar + np.triu(np.full((20, 20), 7.0), 1)
    assert np.array_equal(oracle.chol_adjoint(noisy_L, noisy_b), oracle.chol_adjoint(L, Lbar))
