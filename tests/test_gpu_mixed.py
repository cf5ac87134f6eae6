"""GPU checks of the mixed-precision solve with iterative refinement (through
the C ABI) against the FP64 CPU oracle.

Bar, per right-hand side:
  - the normwise backward error eta = ||b - A x|| / (||A|| ||x|| + ||b||)
    (infinity norms), recomputed here by the oracle with a long-double
    residual, independently of the library's own stopping test, is at most
    the target 1e-12;
  - the forward error against the oracle's FP64 solution stays within what
    the backward errors allow: max|x - x_o| / max|x_o| <=
    2.5 kappa_inf(A) (eta + eta_o), with kappa_inf(A) = ||A|| ||A^{-1}||
    computed here in FP64;
  - refinement really ran (the low-precision first solve misses the target
    on the shift-1e-4 matrices, condition number about 1.3e4);
  - breakdown and non-convergence are reported as documented, and results
    do not depend on the claim order.
Every check runs for both low precisions: FP32 trailing updates, and BF16
updates (each panel value as three BF16 terms, FP32 accumulation).
"""
import numpy as np
import pytest

import oracle
import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TARGET = 1e-12
LOWPS = [1, 2]   # LOWP_FP32, LOWP_BF16


@pytest.fixture(scope="module")
def tc():
    import paper_1402_6601_amd as t
    t.load()
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to the gpu-marked tests")
    return t


def _mixed(tc, A, b, nb, **kw):
    A_d = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    Bc = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()
    rc, iters, berr = tc.solve_mixed_(A_d, Bc, nb, **kw)
    torch.cuda.synchronize()
    return rc, iters, berr, Bc.cpu().numpy().T.copy()


def _kappa_inf(A):
    S = oracle.sym_from_lower(A)
    return float(np.max(np.sum(np.abs(S), axis=1)) * np.max(np.sum(np.abs(np.linalg.inv(S)), axis=1)))


@pytest.mark.parametrize("n,nb,seed,shift,nrhs", [
    (1000, 128, 21, 1e-4, 3),     # ragged last tile
    (1024, 256, 2, 1e-4, 16),     # the mixed workload's matrix family and RHS count, small order
    (513, 512, 22, 1e-4, 1),      # one full tile and a one-row tail
    (999, 160, 23, 1e-4, 5),      # odd order: padded working copy
    (300, 64, 24, 1.0, 2),        # well conditioned
    (17, 16, 25, 1e-4, 4),
    (2048, 512, 26, 1e-4, 16),
])
@pytest.mark.parametrize("lowp", LOWPS)
def test_mixed_reaches_target(tc, n, nb, seed, shift, nrhs, lowp):
    print("case n=%d nb=%d seed=%d shift=%g nrhs=%d lowp=%d" % (n, nb, seed, shift, nrhs, lowp), flush=True)
    A, b = spd_inputs.spd_matrix_and_rhs(n, seed, nrhs=nrhs, shift=shift)
    rc, iters, berr, X = _mixed(tc, A, b, nb, tol=TARGET, maxit=30, lowp=lowp)
    assert rc == 0, (rc, iters, berr)
    assert np.all(berr <= TARGET)
    eta = oracle.solve_backward_error(A, X, b)
    assert np.all(eta <= TARGET), eta
    Xo = oracle.potrs(oracle.cholesky(A), b)
    eta_o = oracle.solve_backward_error(A, Xo, b)
    kap = _kappa_inf(A)
    ex = np.max(np.abs(X - Xo), axis=0) / np.max(np.abs(Xo), axis=0)
    assert np.all(ex <= 2.5 * kap * (eta + eta_o)), (ex, kap, eta, eta_o)
    if shift < 1e-2 and n >= 256:
        assert iters >= 1
    print("  iters=%d max eta=%.3g max e_x=%.3g kappa_inf=%.3g" % (iters, eta.max(), ex.max(), kap), flush=True)


@pytest.mark.parametrize("lowp", LOWPS)
def test_mixed_reported_error_matches_oracle_without_refinement(tc, lowp):
    """maxit = 0: only the low-precision solve; the call reports
    non-convergence and the eta it measured, which the oracle confirms."""
    A, b = spd_inputs.spd_matrix_and_rhs(768, 27, nrhs=4, shift=1e-4)
    rc, iters, berr, X = _mixed(tc, A, b, 128, tol=TARGET, maxit=0, lowp=lowp)
    assert rc == tc.E_NOCONV and iters == 0
    eta = oracle.solve_backward_error(A, X, b)
    assert np.all(eta > TARGET)
    assert np.allclose(berr, eta, rtol=1e-3, atol=1e-18), (berr, eta)
    # the low-precision solution is still close: unit roundoff of FP32 times the condition
    Xo = oracle.potrs(oracle.cholesky(A), b)
    ex = np.max(np.abs(X - Xo), axis=0) / np.max(np.abs(Xo), axis=0)
    assert np.all(ex <= 2.5 * _kappa_inf(A) * (eta + 1e-15))


@pytest.mark.parametrize("lowp", LOWPS)
def test_mixed_bitwise_across_policies(tc, lowp):
    A, b = spd_inputs.spd_matrix_and_rhs(900, 28, nrhs=3, shift=1e-4)
    ref = _mixed(tc, A, b, 128, lowp=lowp)
    for pol, seed in [(tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0), (tc.POLICY_RANDOM, 9)]:
        got = _mixed(tc, A, b, 128, policy=pol, seed=seed, lowp=lowp)
        assert got[0] == ref[0] and got[1] == ref[1]
        assert np.array_equal(got[3], ref[3])


@pytest.mark.parametrize("lowp", LOWPS)
def test_mixed_breakdown_reports_the_minor(tc, lowp):
    A, L0 = spd_inputs.integer_spd(400, seed=29)
    j = 233
    A[j, j] -= 2.0 * L0[j, j] ** 2      # pivot j becomes -L0[j, j]^2: clearly negative
    _, info_o = oracle.potrf(A)
    assert info_o == j + 1
    b = np.ones((400, 2))
    rc, iters, _, X = _mixed(tc, A, b, 64, lowp=lowp)
    assert rc == j + 1 and iters == 0
    assert np.array_equal(X, b)          # B untouched


def test_mixed_fallback_equals_fp64_path(tc):
    A, b = spd_inputs.spd_matrix_and_rhs(640, 30, nrhs=2, shift=1e-4)
    A_d = torch.from_numpy(A).cuda()
    X, info = tc.solve_mixed(A_d, torch.from_numpy(b).cuda(), 128, maxit=0, fallback=True)
    assert info["fallback"] and info["rc"] == tc.E_NOCONV
    W = A_d.clone()
    assert tc.factor_(W, 128) == 0
    X64 = tc.solve(W, torch.from_numpy(b).cuda(), 128, subst=True)
    assert torch.equal(X, X64)
    assert np.all(oracle.solve_backward_error(A, X.cpu().numpy(), b) <= 1e-15)


def test_mixed_degenerate_sizes(tc):
    e = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    rc, iters, berr = tc.solve_mixed_(e, torch.zeros((3, 0), dtype=torch.float64, device="cuda"), 16)
    assert rc == 0 and iters == 0 and np.all(berr == 0)
    A, _ = spd_inputs.spd_matrix_and_rhs(50, 31, nrhs=1)
    A_d = torch.from_numpy(A).cuda()
    rc, iters, berr = tc.solve_mixed_(A_d, torch.zeros((0, 50), dtype=torch.float64, device="cuda"), 16)
    assert rc == 0 and iters == 0
    # n = 1
    A1 = np.array([[4.0]])
    rc, iters, berr, X = _mixed(tc, A1, np.array([[2.0]]), 16)
    assert rc == 0 and abs(X[0, 0] - 0.5) <= 1e-15


def test_bf16_updates_keep_fp32_accuracy(tc):
    """The BF16 path's three-term products keep the updates at FP32 accuracy:
    the backward error of the first low-precision solution (no refinement)
    is of the same size as with FP32 updates (a one-term BF16 product would
    leave it about 2^16 times larger), and the BF16 path needs at most one
    correction more than the FP32 one to reach the target."""
    A, b = spd_inputs.spd_matrix_and_rhs(2048, 34, nrhs=4, shift=1e-4)
    _, _, _, X32 = _mixed(tc, A, b, 512, lowp=1, maxit=0)
    _, _, _, X16 = _mixed(tc, A, b, 512, lowp=2, maxit=0)
    e32 = oracle.solve_backward_error(A, X32, b)
    e16 = oracle.solve_backward_error(A, X16, b)
    print("first-solve eta: fp32 %.3g, bf16 %.3g" % (e32.max(), e16.max()), flush=True)
    assert e16.max() <= 4.0 * e32.max(), (e16, e32)
    _, it32, _, _ = _mixed(tc, A, b, 512, lowp=1)
    rc, it16, _, X = _mixed(tc, A, b, 512, lowp=2)
    assert rc == 0 and it16 <= it32 + 1, (it32, it16)
    assert np.all(oracle.solve_backward_error(A, X, b) <= TARGET)
