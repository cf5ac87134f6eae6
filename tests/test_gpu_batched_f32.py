"""GPU checks of the batched FP32 launch (tchol_factor_solve_batched_f32,
through the C ABI) against the CPU oracle, system by system.

The systems are stored in FP32 (the inputs rounded once); the oracle works
in FP64 on exactly those rounded values.  Bar, per system: the scaled
backward error of the returned FP32 factor, ||A - L L^T||_F /
(n eps32 ||A||_F) with eps32 = 2^-23, at most 10; the solution's
normwise-max error against the oracle's FP64 solution of the same rounded
system at most cond(A) * 1e-5; the oracle's info for a system that is not
positive definite while the others complete; identical results under every
claim order.
"""
import numpy as np
import pytest

import oracle
import spd_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -23


@pytest.fixture(scope="module")
def tc():
    import paper_1402_6601_amd as t
    t.load()
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to the gpu-marked tests")
    return t


def _run(tc, As, bs, nb, **kw):
    """Pack in FP32, run one launch, unpack: (info, [A32_i], [b32_i], [L_i], [X_i]) in float64."""
    Af, ao, lda, Bf, bo = spd_inputs.pack_batched(As, bs, align=4, pad=3, dtype=np.float32)
    n = [a.shape[0] for a in As]
    nrhs = bs[0].shape[1] if bs else 0
    A_d = torch.from_numpy(Af).cuda()
    B_d = torch.from_numpy(Bf).cuda()
    info = tc.factor_solve_batched_f32_(A_d, ao, lda, B_d, bo, n, nb, nrhs, **kw)
    torch.cuda.synchronize()
    Ah, Bh = A_d.cpu().numpy().astype(np.float64), B_d.cpu().numpy().astype(np.float64)
    A32s, b32s, Ls, Xs = [], [], [], []
    for i, m in enumerate(n):
        A32s.append(Af[ao[i]:ao[i] + m * lda[i]].reshape(m, lda[i])[:, :m].astype(np.float64))
        b32s.append(Bf[bo[i]:bo[i] + m * nrhs].reshape(nrhs, m).T.astype(np.float64))
        raw = Ah[ao[i]:ao[i] + m * lda[i]].reshape(m, lda[i])[:, :m]
        Ls.append(np.tril(raw.T))
        Xs.append(Bh[bo[i]:bo[i] + m * nrhs].reshape(nrhs, m).T)
    return info, A32s, b32s, Ls, Xs


def _nb_single(n):
    return max(16, min(512, -(-n // 16) * 16))


SIZES = [1, 16, 17, 100, 128, 255, 300, 511, 512, 513, 700, 33, 64, 250]


def _check(A32, b32, L, X):
    n = A32.shape[0]
    S = oracle.sym_from_lower(A32)
    beta = np.linalg.norm(S - L @ L.T) / (n * EPS32 * np.linalg.norm(S))
    assert beta <= 10.0, beta
    if b32.shape[1]:
        Xo = oracle.potrs(oracle.cholesky(A32), b32)
        cond = np.linalg.cond(S)
        ex = np.max(np.abs(X - Xo)) / np.max(np.abs(Xo))
        assert ex <= cond * 1e-5, (ex, cond)
    return beta


def test_batched_f32_matches_oracle(tc):
    _, As, bs = spd_inputs.batched_systems(len(SIZES), 31, 4, sizes=SIZES)
    nb = [_nb_single(n) if n <= 512 else (128 if n < 600 else 256) for n in SIZES]
    nb[SIZES.index(33)] = 16
    nb[SIZES.index(250)] = 64
    info, A32s, b32s, Ls, Xs = _run(tc, As, bs, nb)
    assert np.all(info == 0)
    worst = 0.0
    for A32, b32, L, X in zip(A32s, b32s, Ls, Xs):
        worst = max(worst, _check(A32, b32, L, X))
    print("max beta32 %.3f" % worst, flush=True)


def test_batched_f32_failure_stays_in_its_system(tc):
    sizes = [200, 300, 64, 129]
    _, As, bs = spd_inputs.batched_systems(len(sizes), 32, 4, sizes=sizes)
    A1, L0 = spd_inputs.integer_spd(300, seed=7)
    j = 137
    A1[j, j] -= 2.0 * L0[j, j] ** 2            # pivot j clearly negative
    _, info_o = oracle.potrf(A1.astype(np.float32).astype(np.float64))
    assert info_o == j + 1
    As[1] = A1
    nb = [_nb_single(200), 128, 64, _nb_single(129)]
    info, A32s, b32s, Ls, Xs = _run(tc, As, bs, nb)
    assert list(info) == [0, j + 1, 0, 0]
    for s in (0, 2, 3):
        _check(A32s[s], b32s[s], Ls[s], Xs[s])


def test_batched_f32_one_tile_compact(tc):
    """Every system one tile: the FP64 copies are factored and solved by the
    compact FP64 instance (two workgroups per compute unit, the forward solve
    riding along the factorization); one system fails and stays alone."""
    sizes = [1, 17, 100, 128, 129, 255, 300, 450, 511, 512, 200]
    _, As, bs = spd_inputs.batched_systems(len(sizes), 35, 4, sizes=sizes)
    A1, L0 = spd_inputs.integer_spd(200, seed=9)
    j = 61
    A1[j, j] -= 2.0 * L0[j, j] ** 2
    _, info_o = oracle.potrf(A1.astype(np.float32).astype(np.float64))
    assert info_o == j + 1
    As[-1] = A1
    info, A32s, b32s, Ls, Xs = _run(tc, As, bs, [_nb_single(n) for n in sizes])
    assert list(info) == [0] * (len(sizes) - 1) + [j + 1]
    for s in range(len(sizes) - 1):
        _check(A32s[s], b32s[s], Ls[s], Xs[s])


def test_batched_f32_bitwise_across_policies(tc):
    sizes = [400, 37, 600, 128, 250]
    _, As, bs = spd_inputs.batched_systems(len(sizes), 33, 3, sizes=sizes)
    nb = [_nb_single(400), 16, 128, 128, 64]
    ref = _run(tc, As, bs, nb)
    for pol, seed in [(tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0), (tc.POLICY_RANDOM, 5)]:
        got = _run(tc, As, bs, nb, policy=pol, seed=seed)
        assert np.array_equal(got[0], ref[0])
        assert all(np.array_equal(a, b) for a, b in zip(got[3], ref[3]))
        assert all(np.array_equal(a, b) for a, b in zip(got[4], ref[4]))


def test_batched_f32_factor_only_empty_and_layout(tc):
    _, As, bs = spd_inputs.batched_systems(3, 34, 0, sizes=[100, 0, 50])
    info, A32s, _, Ls, _ = _run(tc, As, bs, [112, 16, 64])
    assert np.all(info == 0)
    for A32, L in zip(A32s, Ls):
        if A32.shape[0]:
            S = oracle.sym_from_lower(A32)
            assert np.linalg.norm(S - L @ L.T) / (A32.shape[0] * EPS32 * np.linalg.norm(S)) <= 10.0
    e = torch.zeros(4, dtype=torch.float32, device="cuda")
    assert len(tc.factor_solve_batched_f32_(e, [], [], e, [], [], [], 4)) == 0
    # a leading dimension without the three padding rows is rejected before any launch
    A = torch.zeros(64 * 64, dtype=torch.float32, device="cuda")
    with pytest.raises(tc.TcholError):
        tc.factor_solve_batched_f32_(A, [0], [64], A, [0], [64], [64], 1)


def test_batched_f32_config5_full_size(tc):
    """The FP32 batch at its full size (4096 systems of orders uniform in
    [16, 512], seed 4, 4 right-hand sides, tuned table, one launch): every
    system's factor within 10 n eps32 ||A||_F of its FP32 matrix and every
    solution's normwise backward error at most 1e-6, both computed on the
    device in FP64 as checkers."""
    from paper_1402_6601_amd import autotune
    print("case: 4096 FP32 systems, seed 4, 4 RHS, tuned table", flush=True)
    ns, A0, a_off, lda, B0, b_off = spd_inputs.batched_systems_device(4096, 4, 4, align=4, pad=3, fp32=True)
    nb = autotune.tile_sizes(ns)
    A, B = A0.clone(), B0.clone()
    info = tc.factor_solve_batched_f32_(A, a_off, lda, B, b_off, ns, nb, 4)
    torch.cuda.synchronize()
    assert np.all(info == 0)
    worst_beta, worst_eta = 0.0, 0.0
    for n, o, l, ob in zip(ns, a_off, lda, b_off):
        n, o, l, ob = int(n), int(o), int(l), int(ob)
        S = A0[o:o + n * l].view(n, l)[:, :n].double()
        L = torch.tril(A[o:o + n * l].view(n, l)[:, :n].t().double())
        beta = float(torch.linalg.norm(S - L @ L.t().contiguous()) / (n * EPS32 * torch.linalg.norm(S)))
        b = B0[ob:ob + n * 4].view(4, n).t().double()
        x = B[ob:ob + n * 4].view(4, n).t().double()
        r = b - S @ x.contiguous()
        an = float(torch.max(torch.sum(torch.abs(S), dim=1)))
        eta = torch.max(torch.abs(r), dim=0).values / (an * torch.max(torch.abs(x), dim=0).values +
                                                      torch.max(torch.abs(b), dim=0).values)
        worst_beta = max(worst_beta, beta)
        worst_eta = max(worst_eta, float(torch.max(eta)))
    print("worst beta32 %.3f, worst eta %.3e" % (worst_beta, worst_eta), flush=True)
    assert worst_beta <= 10.0
    assert worst_eta <= 1e-6
