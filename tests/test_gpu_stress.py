"""Bounded determinism stress of the persistent scheduler's publish protocol
(write-through stores, a completion counter, an acquire by the reader): about
200 factorizations at n = 2048 ... 8192 under every claim policy (random
orders with fresh seeds), each factor bitwise equal to the first one of its
size; a stale read anywhere would change bits.  Stops at the first mismatch."""
import numpy as np
import pytest

import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [(2048, 256, 80), (4096, 512, 60), (8192, 512, 60)]


@pytest.mark.parametrize("n,nb,reps", CASES)
def test_factor_bitwise_under_repeated_launches(n, nb, reps):
    import paper_1402_6601_amd as tc
    tc.load()
    A0, _ = spd_inputs.spd_matrix_device(n, 90 + n // 1024, 1.0, device="cuda")
    ref = A0.clone()
    assert tc.factor_(ref, nb) == 0
    W = torch.empty_like(A0)
    policies = [tc.POLICY_LIST, tc.POLICY_RANK, tc.POLICY_FIFO, tc.POLICY_RANDOM]
    for r in range(reps):
        W.copy_(A0)
        pol = policies[r % 4]
        assert tc.factor_(W, nb, policy=pol, seed=1000 + r) == 0
        if not torch.equal(W, ref):
            diff = (W - ref).abs().max().item()
            pytest.fail("n=%d nb=%d repetition %d policy %d: factor differs (max %.3e)" % (n, nb, r, pol, diff))
    print("n=%d nb=%d: %d factorizations bitwise equal" % (n, nb, reps), flush=True)


def test_merged_bitwise_under_repeated_launches():
    import paper_1402_6601_amd as tc
    tc.load()
    n, nb, nrhs = 4096, 512, 16
    A0, rng = spd_inputs.spd_matrix_device(n, 95, 1.0, device="cuda")
    B0 = torch.from_numpy(np.ascontiguousarray(spd_inputs.rhs(rng, n, nrhs).T)).cuda()
    W, X = A0.clone(), B0.clone()
    assert tc.factor_solve_(W, X, nb) == 0
    W2, X2 = torch.empty_like(W), torch.empty_like(X)
    for r in range(24):
        W2.copy_(A0)
        X2.copy_(B0)
        assert tc.factor_solve_(W2, X2, nb, policy=r % 4, seed=77 + r) == 0
        assert torch.equal(W2, W) and torch.equal(X2, X), "repetition %d" % r
