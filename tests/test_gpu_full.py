"""Parity at the benchmark's full size (n = 32768, nb = 512, 16 right-hand
sides, seed 1), on the launch bench.py times: tchol_factor_solve, the
factorization and the solve merged into one DAG in one launch, with the
default claim order.  The oracle cannot factor the whole matrix in test time,
so the checks are ones it can compute one by one or that hold at any size:
- the merged launch's L and X are bitwise equal to those of the factorization
  (with the same inverse-applying TRSMs) and the solve launched one after the
  other (the same DAG semantics);
- the leading m x m block of L equals the oracle's factor of the leading
  principal m x m block of A (an exact sub-result of the Cholesky factor);
- the whole factor's scaled backward error ||A - L L^T||_F / (n eps ||A||_F)
  is at most 10 (the product L L^T is formed by torch in FP64, as a checker
  only);
- sampled entries of L L^T reproduce A, accumulated in long double;
- sampled rows of the solve's residual, accumulated in long double, give a
  normwise backward error at FP64 rounding level for every right-hand side.
"""
import numpy as np
import pytest

import oracle
import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, NB, NRHS, SEED = 32768, 512, 16, 1


@pytest.fixture(scope="module")
def merged():
    import paper_1402_6601_amd as tc
    tc.load()
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to the gpu-marked tests")
    print("generating n=%d" % N, flush=True)
    A0, rng = spd_inputs.spd_matrix_device(N, SEED, 1.0, device="cuda")
    B = torch.from_numpy(spd_inputs.rhs(rng, N, NRHS)).cuda()      # (n, nrhs) row-major
    Bc0 = B.t().contiguous()                                        # column-major B
    W = A0.clone()
    Xc = Bc0.clone()
    print("merged factor + solve launch", flush=True)
    info = tc.factor_solve_(W, Xc, NB)
    assert info == 0
    torch.cuda.synchronize()
    return tc, A0, W, B, Bc0, Xc


def test_merged_equals_two_launches_bitwise(merged):
    tc, A0, W, _, Bc0, Xc = merged
    W2 = A0.clone()
    print("factor, then solve, as two launches", flush=True)
    assert tc.factor_(W2, NB, inv_trsm=True) == 0
    X2 = Bc0.clone()
    tc.solve_(W2, X2, NB)
    torch.cuda.synchronize()
    assert torch.equal(W, W2)
    assert torch.equal(Xc, X2)
    del W2, X2
    torch.cuda.empty_cache()


def test_leading_block_matches_oracle(merged):
    _, A0, W, _, _, _ = merged
    m = 4096
    lead = A0[:m, :m].cpu().numpy()
    F, info = oracle.potrf(np.ascontiguousarray(lead.T))
    assert info == 0
    Lg = np.tril(W[:m, :m].cpu().numpy().T)
    assert oracle.factor_error(Lg, F) <= 1e-10


def test_full_backward_error(merged):
    _, A0, W, _, _, _ = merged
    Lt = torch.triu(W)                       # the row-major view holds L^T in its upper triangle
    P = torch.mm(Lt.t().contiguous(), Lt)    # L L^T
    del Lt
    P.sub_(A0)
    beta = float(torch.linalg.matrix_norm(P).item()) / (N * 2.0 ** -52 * float(torch.linalg.matrix_norm(A0).item()))
    del P
    torch.cuda.empty_cache()
    print("scaled backward error %.3e" % beta, flush=True)
    assert beta <= 10.0


def test_sampled_reconstruction(merged):
    _, A0, W, _, _, _ = merged
    rng = np.random.default_rng(7)
    amax = float(A0.abs().max().item())
    worst = 0.0
    for _ in range(96):
        i = int(rng.integers(0, N))
        j = int(rng.integers(0, i + 1))
        li = W[: i + 1, i].cpu().numpy().astype(np.longdouble)   # row i of L
        lj = W[: j + 1, j].cpu().numpy().astype(np.longdouble)
        s = float(np.sum(li[: j + 1] * lj[: j + 1]))
        worst = max(worst, abs(s - float(A0[j, i].item())))
    assert worst / (N * 2.0 ** -52 * amax) <= 10.0


def test_sampled_solve_backward_error(merged):
    _, A0, _, B, _, Xc = merged
    rng = np.random.default_rng(8)
    rows = rng.choice(N, 64, replace=False)
    Ar = A0[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.longdouble)   # rows of symmetric A
    Xh = Xc.t().cpu().numpy()
    Bh = B.cpu().numpy()
    R = Bh[rows].astype(np.longdouble) - Ar @ Xh.astype(np.longdouble)
    anorm = float(A0.abs().sum(dim=1).max().item())
    den = anorm * np.max(np.abs(Xh), axis=0) + np.max(np.abs(Bh), axis=0)
    eta = np.max(np.abs(R).astype(np.float64), axis=0) / den
    assert eta.shape == (NRHS,)
    assert np.all(eta <= 1e-14), eta
