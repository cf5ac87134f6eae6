"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bar: the normwise-max entry error of L, max|L_gpu - L| / max|L|, at most
1e-10 (the FP64 target; the expected value is about 1e-15 for these
well-conditioned matrices), bit-exact results on integer inputs whose exact
factor is known, the oracle's info on breakdown, and bitwise reproducibility
across runs and claim orders (every tile sees its updates in a fixed order).
"""
import numpy as np
import pytest

import oracle
import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def tc():
    import paper_1402_6601_amd as t
    t.load()
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to the gpu-marked tests")
    return t


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _factor(tc, A_np, nb, **kw):
    """Factor on the GPU; returns (L lower as numpy, info, raw row-major buffer on host)."""
    W = _dev(A_np)
    info = tc.factor_(W, nb, **kw)
    torch.cuda.synchronize()
    raw = W.cpu().numpy()
    return np.tril(raw.T), info, raw


@pytest.mark.parametrize("n,nb,seed", [(1024, 128, 0), (1000, 128, 5), (513, 512, 6), (300, 64, 7),
                                       (17, 16, 8), (1, 16, 9), (100, 512, 10), (640, 160, 11), (4096, 512, 12)])
def test_factor_matches_oracle(tc, n, nb, seed):
    print("case n=%d nb=%d seed=%d" % (n, nb, seed), flush=True)
    A, _ = spd_inputs.spd_matrix(n, seed, shift=1.0)
    L, info, _ = _factor(tc, A, nb)
    assert info == 0
    Lo = oracle.cholesky(A)
    err = oracle.factor_error(L, Lo)
    assert err <= TOL, err
    assert oracle.backward_error(A, L) <= 10.0


def test_config1_factor_and_solve(tc):
    """n=1024, nb=128, A = B B^T/n + I (seed 0), one right-hand side."""
    A, b = spd_inputs.spd_matrix_and_rhs(1024, 0, nrhs=1)
    W = _dev(A)
    assert tc.factor_(W, 128) == 0
    x = tc.solve(W, _dev(b[:, 0]), 128).cpu().numpy()
    L = np.tril(W.cpu().numpy().T)
    Lo = oracle.cholesky(A)
    assert oracle.factor_error(L, Lo) <= TOL
    xo = oracle.potrs(Lo, b[:, 0])
    assert np.max(np.abs(x - xo)) / np.max(np.abs(xo)) <= TOL
    assert oracle.solve_backward_error(A, x, b[:, 0])[0] <= 1e-15


@pytest.mark.parametrize("n,nb,nrhs", [(1000, 128, 16), (512, 64, 3), (700, 512, 20), (33, 16, 1), (1000, 256, 17),
                                         (600, 384, 5), (500, 144, 7), (2048, 512, 16)])
def test_solve_matches_oracle(tc, n, nb, nrhs):
    A, B = spd_inputs.spd_matrix_and_rhs(n, n + nrhs, nrhs=nrhs)
    W = _dev(A)
    assert tc.factor_(W, nb) == 0
    X = tc.solve(W, _dev(B), nb).cpu().numpy()
    Xo = oracle.potrs(oracle.cholesky(A), B)
    assert np.max(np.abs(X - Xo)) / np.max(np.abs(Xo)) <= TOL
    assert np.all(oracle.solve_backward_error(A, X, B) <= 1e-15)


@pytest.mark.parametrize("n,nb", [(64, 16), (300, 64), (640, 128)])
def test_exact_integer_recovery(tc, n, nb):
    A, L0 = spd_inputs.integer_spd(n, seed=n)
    L, info, _ = _factor(tc, A, nb)
    assert info == 0
    assert np.array_equal(L, L0)
    b, x0 = spd_inputs.integer_rhs(A, 4, seed=n)
    W = _dev(A)
    assert tc.factor_(W, nb) == 0
    # substitution keeps every intermediate an integer (the 4 x 4 inverses of
    # its micro-steps are exact with power-of-two pivots); explicit inverses
    # of whole tiles of such a factor are not representable
    x = tc.solve(W, _dev(b), nb, subst=True).cpu().numpy()
    assert np.array_equal(x, x0)


def test_upper_triangle_untouched(tc):
    A, _ = spd_inputs.spd_matrix(700, 3)
    # the library reads the column-major lower triangle = row-major upper triangle;
    # poison the other half and check that it is neither read nor written
    P = np.array(A)
    P[np.tril_indices(700, -1)] = np.nan
    L, info, raw = _factor(tc, P, 128)
    assert info == 0
    assert oracle.factor_error(L, oracle.cholesky(A)) <= TOL
    assert np.all(np.isnan(raw[np.tril_indices(700, -1)]))


@pytest.mark.parametrize("j", [0, 37, 127, 128, 300, 639])
def test_breakdown_info(tc, j):
    A, L0 = spd_inputs.integer_spd(640, seed=2)
    A[j, j] -= L0[j, j] ** 2
    _, info_o = oracle.potrf(A)
    assert info_o == j + 1
    _, info, _ = _factor(tc, A, 128)
    assert info == j + 1


def test_nan_pivot_info(tc):
    A, _ = spd_inputs.spd_matrix(512, 4)
    A[200, 200] = np.nan
    _, info_o = oracle.potrf(A)
    _, info, _ = _factor(tc, A, 128)
    assert info == info_o == 201


def test_bitwise_determinism_across_runs_and_policies(tc):
    A, _ = spd_inputs.spd_matrix(1536, 13)
    ref, info, _ = _factor(tc, A, 128)
    assert info == 0
    for _ in range(4):
        L, info, _ = _factor(tc, A, 128)
        assert info == 0 and np.array_equal(L, ref)
    for pol, seed in [(tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0), (tc.POLICY_RANDOM, 1), (tc.POLICY_RANDOM, 2)]:
        L, info, _ = _factor(tc, A, 128, policy=pol, seed=seed)
        assert info == 0 and np.array_equal(L, ref)


def test_zero_size_and_bad_args(tc):
    W = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    assert tc.factor_(W, 128) == 0
    W = _dev(np.eye(4))
    with pytest.raises(tc.TcholError):
        tc.factor_(W, 100)  # nb not a multiple of 16


def test_wait_bound_turns_into_timeout(tc):
    """A bound of 1 us on each dependency wait makes the first real wait expire:
    the kernel must then drain and report TCHOL_E_TIMEOUT instead of hanging."""
    A, _ = spd_inputs.spd_matrix(2048, 14)
    W = _dev(A)
    rc = tc.factor_(W, 128, wait_limit_us=1, check=False)
    assert rc == tc.E_TIMEOUT
    # the library stays usable afterwards
    W = _dev(A)
    assert tc.factor_(W, 128) == 0


def test_kernel_time_reported(tc):
    A, _ = spd_inputs.spd_matrix(1024, 15)
    W = _dev(A)
    rc, ms = tc.factor_(W, 128, want_kernel_ms=True)
    assert rc == 0 and ms > 0.0


@pytest.mark.parametrize("subst", [False, True])
@pytest.mark.parametrize("n,nb,nrhs,seed", [(1000, 128, 5, 40), (1024, 256, 16, 41), (999, 160, 3, 42),
                                            (513, 512, 1, 43), (17, 16, 2, 44), (300, 64, 0, 45)])
def test_factor_solve_one_launch_equals_two(tc, n, nb, nrhs, seed, subst):
    """The merged factor + solve launch gives bitwise the results of the two
    separate launches (every tile sees the same updates in the same order),
    with the diagonal tiles' inverses (computed in either launch by the same
    tasks, and applied by the TRSMs too: the factor launch with inv_trsm) and
    with substitution everywhere."""
    print("case n=%d nb=%d nrhs=%d subst=%d" % (n, nb, nrhs, subst), flush=True)
    A, b = spd_inputs.spd_matrix_and_rhs(n, seed, nrhs=max(nrhs, 1))
    b = b[:, :nrhs]
    W1, W2 = _dev(A), _dev(A)
    B1 = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()
    B2 = B1.clone()
    assert tc.factor_solve_(W1, B1, nb, subst=subst) == 0
    assert tc.factor_(W2, nb, inv_trsm=not subst) == 0
    if nrhs:
        assert tc.solve_(W2, B2, nb, subst=subst) == 0
    torch.cuda.synchronize()
    assert torch.equal(W1, W2) and torch.equal(B1, B2)
    L = np.tril(W1.cpu().numpy().T)
    assert oracle.factor_error(L, oracle.cholesky(A)) <= TOL
    if nrhs:
        Xo = oracle.potrs(oracle.cholesky(A), b)
        X = B1.cpu().numpy().T
        assert np.max(np.abs(X - Xo)) / np.max(np.abs(Xo)) <= TOL


def test_factor_solve_one_launch_integer_and_breakdown(tc):
    A, L0 = spd_inputs.integer_spd(300, seed=46)
    b, x0 = spd_inputs.integer_rhs(A, 3, seed=46)
    W = _dev(A)
    Bc = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()
    assert tc.factor_solve_(W, Bc, 64, subst=True) == 0
    assert np.array_equal(np.tril(W.cpu().numpy().T), L0)
    assert np.array_equal(Bc.cpu().numpy().T, x0)
    j = 150
    A[j, j] -= L0[j, j] ** 2
    W = _dev(A)
    Bc = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()
    assert tc.factor_solve_(W, Bc, 64) == j + 1


@pytest.mark.parametrize("n,nb,shift,seed", [(1000, 128, 1e-6, 47), (1024, 512, 1e-8, 48), (777, 96, 1e-4, 49)])
def test_inverse_solve_backward_error(tc, n, nb, shift, seed):
    """The solve through the diagonal tiles' explicit inverses on ill-conditioned
    SPD systems (cond(A) about 1.3 / shift): its normwise backward error stays
    within 64 sqrt(cond(A)) eps (cond(L_kk)^2 <= cond(A) for the Cholesky
    factor's diagonal tiles), and substitution's within 16 eps."""
    print("case n=%d nb=%d shift=%g" % (n, nb, shift), flush=True)
    A, b = spd_inputs.spd_matrix_and_rhs(n, seed, nrhs=4, shift=shift)
    W = _dev(A)
    assert tc.factor_(W, nb) == 0
    eps = 2.0 ** -52
    kappa = 1.4 / shift
    for subst, bound in ((False, 64 * np.sqrt(kappa) * eps), (True, 16 * eps)):
        x = tc.solve(W, _dev(b), nb, subst=subst).cpu().numpy()
        berr = np.max(oracle.solve_backward_error(A, x, b))
        print("  subst=%d backward error %.3g (bound %.3g)" % (subst, berr, bound), flush=True)
        assert berr <= bound
