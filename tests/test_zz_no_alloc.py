"""tchol_factor_solve_noalloc: the merged factor + solve launch with its
scheduler scratch in the library's fixed per-GPU array, for callers that
cannot allocate.  Through the C ABI, on two calls in a row (the second on a
smaller problem, so it meets the first call's leftovers in the array), its
factor and solution must be bitwise equal to those of tchol_factor_solve
with a caller workspace and substitution in the solve (the option it runs
with), and within the oracle tolerance of the oracle."""
import numpy as np
import pytest

import oracle
import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(tc, n, nb, nrhs, seed):
    A, B = spd_inputs.spd_matrix_and_rhs(n, seed, nrhs=nrhs)
    W1 = torch.from_numpy(A).cuda()
    X1 = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    W2, X2 = W1.clone(), X1.clone()
    print("noalloc case n=%d nb=%d nrhs=%d seed=%d" % (n, nb, nrhs, seed), flush=True)
    assert tc.factor_solve_(W1, X1, nb, subst=True) == 0
    assert tc.factor_solve_noalloc_(W2, X2, nb) == 0
    torch.cuda.synchronize()
    assert torch.equal(W1, W2)
    assert torch.equal(X1, X2)
    return A, B, W2, X2


def test_noalloc_equals_workspace_launch_twice():
    import paper_1402_6601_amd as tc
    tc.load()
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to the gpu-marked tests")
    # first a larger problem, then a smaller one over the first call's leftovers
    for n, nb, nrhs, seed in [(4100, 512, 5, 61), (1000, 128, 3, 62)]:
        A, B, W, X = _case(tc, n, nb, nrhs, seed)
        if n <= 1000:
            Lo = oracle.cholesky(A)
            assert oracle.factor_error(np.tril(W.cpu().numpy().T), Lo) <= 1e-10
            xo = oracle.potrs(Lo, B)
            xg = X.cpu().numpy().T
            assert np.max(np.abs(xg - xo)) / np.max(np.abs(xo)) <= 1e-10


def test_noalloc_breakdown_and_limit():
    import paper_1402_6601_amd as tc
    tc.load()
    # a non-SPD leading minor: the same info as the workspace launch
    n, nb, j = 600, 128, 300
    A, _ = spd_inputs.spd_matrix_and_rhs(n, 63, nrhs=1)
    A[j, j] = -1.0
    W1 = torch.from_numpy(A).cuda()
    W2 = W1.clone()
    X1 = torch.zeros(1, n, dtype=torch.float64, device="cuda")
    X2 = X1.clone()
    assert tc.factor_solve_(W1, X1, nb, subst=True) == j + 1
    assert tc.factor_solve_noalloc_(W2, X2, nb) == j + 1
    # beyond the fixed array: refused before any device work, nothing touched
    big = torch.zeros(4, dtype=torch.float64, device="cuda")
    lib = tc.load()
    import ctypes
    rc = lib.tchol_factor_solve_noalloc(ctypes.c_void_p(big.data_ptr()), 32768, 256, ctypes.c_void_p(big.data_ptr()),
                                        16, None)
    assert rc == tc.E_SCRATCH
    assert torch.count_nonzero(big).item() == 0
