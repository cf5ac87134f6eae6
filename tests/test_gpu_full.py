"""Parity at the benchmark's full size (n = 32768, nb = 512, 16 RHS), in the
launch configuration bench.py times.  The oracle cannot factor the whole
matrix in test time, so the checks are ones it can compute one by one or that
hold at any size:
- the leading m x m block of L equals the oracle's factor of the leading
  principal m x m block of A (an exact sub-result of the Cholesky factor);
- sampled entries of L L^T reproduce A to the backward-error bound;
- sampled rows of the solve's residual, accumulated in long double, give a
  normwise backward error at FP64 rounding level.
"""
import numpy as np
import pytest

import oracle
import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, NB, NRHS, SEED = 32768, 512, 16, 1


@pytest.fixture(scope="module")
def factored():
    import paper_1402_6601_amd as tc
    tc.load()
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to the gpu-marked tests")
    print("generating n=%d" % N, flush=True)
    A0, rng = spd_inputs.spd_matrix_device(N, SEED, 1.0, device="cuda")
    B = torch.from_numpy(spd_inputs.rhs(rng, N, NRHS)).cuda()
    W = A0.clone()
    print("factoring", flush=True)
    info = tc.factor_(W, NB)
    assert info == 0
    X = tc.solve(W, B, NB)
    torch.cuda.synchronize()
    print("factored", flush=True)
    return tc, A0, W, B, X


def test_leading_block_matches_oracle(factored):
    _, A0, W, _, _ = factored
    m = 4096
    lead = A0[:m, :m].cpu().numpy()
    F, info = oracle.potrf(np.ascontiguousarray(lead.T))
    assert info == 0
    Lg = np.tril(W[:m, :m].cpu().numpy().T)
    assert oracle.factor_error(Lg, F) <= 1e-10


def test_sampled_reconstruction(factored):
    _, A0, W, _, _ = factored
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


def test_sampled_solve_backward_error(factored):
    _, A0, _, B, X = factored
    rng = np.random.default_rng(8)
    rows = rng.choice(N, 64, replace=False)
    Ar = A0[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.longdouble)   # rows of symmetric A
    Xh = X.cpu().numpy()
    Bh = B.cpu().numpy()
    R = Bh[rows].astype(np.longdouble) - Ar @ Xh.astype(np.longdouble)
    anorm = float(A0.abs().sum(dim=1).max().item())
    den = anorm * np.max(np.abs(Xh), axis=0) + np.max(np.abs(Bh), axis=0)
    eta = np.max(np.abs(R).astype(np.float64), axis=0) / den
    assert np.all(eta <= 1e-14), eta
