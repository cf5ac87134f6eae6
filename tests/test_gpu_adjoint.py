"""GPU parity of the Cholesky adjoint (tchol_backward, through the C ABI and
the autograd function) against the CPU oracle.

Bar: max |Abar_gpu - Abar_oracle| / max |Abar_oracle| <= 1e-10 on the same
factor L and upstream Lbar (tril of N(0, 1)); the log-det identity
(Lbar = diag(2 / L_ii) gives A^{-1}) to 1e-10; central finite differences of
the library's own forward factorization at n = 48 (h = 1e-6) to 1e-6 of
max |Abar|; bitwise-equal results under every claim order; the strict upper
triangles of L and Lbar neither read nor written.
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


def _colmajor(M):
    """A device buffer whose column-major reading is M."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(M, dtype=np.float64).T)).cuda()


def _adjoint(tc, L, Lbar, nb, upper_fill=0.0, **kw):
    n = L.shape[0]
    Lb = _colmajor(np.tril(L) + np.triu(np.full((n, n), upper_fill), 1))
    Gb = _colmajor(np.tril(Lbar) + np.triu(np.full((n, n), upper_fill), 1))
    rc = tc.backward_(Lb, Gb, nb, **kw)
    torch.cuda.synchronize()
    assert rc == 0
    raw = Gb.cpu().numpy().T   # column-major reading
    return raw


def _sym_lower(raw):
    low = np.tril(raw)
    return low + np.tril(low, -1).T


@pytest.mark.parametrize("n,nb,seed", [(100, 16, 0), (300, 64, 1), (513, 128, 2), (640, 160, 3), (17, 16, 4),
                                       (1, 16, 5), (1000, 256, 6), (256, 256, 7), (999, 128, 8), (48, 32, 9)])
def test_adjoint_matches_oracle(tc, n, nb, seed):
    print("case n=%d nb=%d seed=%d" % (n, nb, seed), flush=True)
    A, rng = spd_inputs.spd_matrix(n, seed)
    L = oracle.cholesky(A)
    Lbar = spd_inputs.lower_upstream(rng, n)
    got = _sym_lower(_adjoint(tc, L, Lbar, nb))
    ref = oracle.chol_adjoint(L, Lbar)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= TOL, err


def test_logdet_gradient_is_inverse(tc):
    n, nb = 500, 128
    A, _ = spd_inputs.spd_matrix(n, 10)
    L = oracle.cholesky(A)
    got = _sym_lower(_adjoint(tc, L, np.diag(2.0 / np.diag(L)), nb))
    inv = np.linalg.inv(A)
    assert np.max(np.abs(got - inv)) / np.max(np.abs(inv)) <= TOL


def test_finite_differences_through_autograd(tc):
    n, nb, h = 48, 16, 1e-6
    A, rng = spd_inputs.spd_matrix(n, 3)
    Lbar = spd_inputs.lower_upstream(rng, n)
    A_d = torch.from_numpy(A).cuda().requires_grad_(True)
    W = torch.from_numpy(Lbar).cuda()
    L = tc.cholesky(A_d, nb)
    (L * W).sum().backward()
    G = A_d.grad.cpu().numpy()
    assert np.array_equal(G, G.T)

    def f(M):
        Lm, info = tc.factor(torch.from_numpy(M).cuda(), nb)
        assert info == 0
        return float((Lm * W).sum().item())

    scale = np.max(np.abs(G))
    rs = np.random.default_rng(1)
    pairs = [(i, i) for i in range(0, n, 9)] + [tuple(sorted(rs.integers(0, n, 2), reverse=True)) for _ in range(24)]
    for i, j in pairs:
        S = np.zeros((n, n))
        S[i, j] += 1.0
        if i != j:
            S[j, i] += 1.0
        fd = (f(A + h * S) - f(A - h * S)) / (2 * h)
        want = G[i, j] if i == j else 2.0 * G[i, j]
        assert abs(fd - want) <= 1e-6 * scale, (i, j, fd, want)


def test_adjoint_bitwise_across_policies(tc):
    A, rng = spd_inputs.spd_matrix(700, 11)
    L = oracle.cholesky(A)
    Lbar = spd_inputs.lower_upstream(rng, 700)
    ref = _adjoint(tc, L, Lbar, 128)
    for pol, seed in [(tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0), (tc.POLICY_RANDOM, 3)]:
        got = _adjoint(tc, L, Lbar, 128, policy=pol, seed=seed)
        assert np.array_equal(got, ref)


def test_adjoint_upper_triangles_untouched(tc):
    n, nb = 200, 64
    A, rng = spd_inputs.spd_matrix(n, 12)
    L = oracle.cholesky(A)
    Lbar = spd_inputs.lower_upstream(rng, n)
    raw = _adjoint(tc, L, Lbar, nb, upper_fill=np.nan)
    assert np.all(np.isnan(np.triu(raw, 1)[np.triu_indices(n, 1)]))
    got = _sym_lower(np.where(np.isnan(raw), 0.0, raw))
    ref = oracle.chol_adjoint(L, Lbar)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= TOL


def test_adjoint_degenerate_and_bad_args(tc):
    e = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    assert tc.backward_(e, e.clone(), 16) == 0
    x = torch.eye(8, dtype=torch.float64, device="cuda")
    with pytest.raises(tc.TcholError):
        tc.backward_(x, x.clone(), 24)
    with pytest.raises(ValueError):
        tc.backward_(x, torch.zeros((8, 7), dtype=torch.float64, device="cuda"), 16)
