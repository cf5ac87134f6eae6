"""GPU parity of the batched factor + solve launch (through the C ABI) against
the CPU oracle, system by system.

Bar, per system: the normwise-max entry error of L at most 1e-10 and of the
solution at most 1e-10 (FP64), the oracle's info for a system that is not
positive definite while every other system of the batch completes, exact
results for integer systems, and bitwise-equal results under every claim
order.  Systems mix single-tile orders (one workgroup each) with multi-tile
ones (their tiles spread over workgroups), ragged edge tiles, and both the
16-byte (even leading dimension) and 4-byte transfer paths.
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


def _run(tc, As, bs, nb, align=2, **kw):
    """Pack, run one batched launch, unpack: returns (info, [L_i], [X_i])."""
    Af, ao, lda, Bf, bo = spd_inputs.pack_batched(As, bs, align)
    A_d = torch.from_numpy(Af).cuda()
    B_d = torch.from_numpy(Bf).cuda()
    n = [a.shape[0] for a in As]
    nrhs = bs[0].shape[1] if bs else 0
    info = tc.factor_solve_batched_(A_d, ao, lda, B_d, bo, n, nb, nrhs, **kw)
    torch.cuda.synchronize()
    Ah, Bh = A_d.cpu().numpy(), B_d.cpu().numpy()
    Ls, Xs = [], []
    for i, m in enumerate(n):
        raw = Ah[ao[i]:ao[i] + m * lda[i]].reshape(m, lda[i])[:, :m]   # row c = column c
        Ls.append(np.tril(raw.T))
        Xs.append(Bh[bo[i]:bo[i] + m * nrhs].reshape(nrhs, m).T)
    return info, Ls, Xs


def _nb_single(n):
    return max(16, min(512, -(-n // 16) * 16))


SIZES = [1, 16, 17, 100, 128, 255, 300, 511, 512, 513, 700, 33, 64, 250]


def _systems(seed, sizes, nrhs=4):
    _, As, bs = spd_inputs.batched_systems(len(sizes), seed, nrhs, sizes=sizes)
    return As, bs


@pytest.mark.parametrize("align", [2, 1])
def test_batched_matches_oracle(tc, align):
    As, bs = _systems(11, SIZES)
    # single-tile systems up to 512; larger ones tiled by 128 / 256; two small
    # systems tiled by 16 to exercise multi-tile DAGs of small orders
    nb = [_nb_single(n) if n <= 512 else (128 if n < 600 else 256) for n in SIZES]
    nb[SIZES.index(33)] = 16
    nb[SIZES.index(250)] = 64
    info, Ls, Xs = _run(tc, As, bs, nb, align=align)
    assert np.all(info == 0)
    for A, b, L, X in zip(As, bs, Ls, Xs):
        Lo = oracle.cholesky(A)
        assert oracle.factor_error(L, Lo) <= TOL
        Xo = oracle.potrs(Lo, b)
        assert np.max(np.abs(X - Xo)) / max(np.max(np.abs(Xo)), 1e-300) <= TOL
        assert np.all(oracle.solve_backward_error(A, X, b) <= 1e-15)


def test_batched_failure_stays_in_its_system(tc):
    sizes = [200, 300, 64, 129]
    As, bs = _systems(12, sizes)
    A1, L0 = spd_inputs.integer_spd(300, seed=5)
    j = 137
    A1[j, j] -= L0[j, j] ** 2
    _, info_o = oracle.potrf(A1)
    assert info_o == j + 1
    As[1] = A1
    nb = [_nb_single(200), 128, 64, _nb_single(129)]
    info, Ls, Xs = _run(tc, As, bs, nb)
    assert list(info) == [0, j + 1, 0, 0]
    for s in (0, 2, 3):
        Lo = oracle.cholesky(As[s])
        assert oracle.factor_error(Ls[s], Lo) <= TOL
        Xo = oracle.potrs(Lo, bs[s])
        assert np.max(np.abs(Xs[s] - Xo)) / np.max(np.abs(Xo)) <= TOL


@pytest.mark.parametrize("align", [2, 1])
def test_batched_single_tile_breakdown(tc, align):
    """Breakdown inside one-tile systems above 128 (one workgroup, panels of
    32 columns in slabs of 256 rows): in the leading and in the trailing 16
    columns of a panel, in the first panel, and in a panel whose rows span
    two slabs; the oracle's info for each, the other systems exact."""
    sizes = [400, 400, 400, 300, 511, 200]
    cols = [37, 50, 5, 290, 20, None]
    As, bs = _systems(13, sizes)
    for s, j in enumerate(cols):
        if j is None:
            continue
        A1, L0 = spd_inputs.integer_spd(sizes[s], seed=20 + s)
        A1[j, j] -= L0[j, j] ** 2
        _, info_o = oracle.potrf(A1)
        assert info_o == j + 1
        As[s] = A1
    nb = [_nb_single(n) for n in sizes]
    info, Ls, Xs = _run(tc, As, bs, nb, align=align)
    assert list(info) == [0 if j is None else j + 1 for j in cols]
    Lo = oracle.cholesky(As[-1])
    assert oracle.factor_error(Ls[-1], Lo) <= TOL
    Xo = oracle.potrs(Lo, bs[-1])
    assert np.max(np.abs(Xs[-1] - Xo)) / np.max(np.abs(Xo)) <= TOL


@pytest.mark.parametrize("align", [2, 1])
def test_batched_shared_factorization(tc, align):
    """One-tile systems whose factorization several workgroups share
    (tchol_opts.wgs, the tile's sub-block pool) match the oracle; a breakdown
    inside a shared factorization gives the oracle's info and stays in its
    system; wgs on systems of 128 or less changes nothing."""
    sizes = [129, 200, 300, 512, 400, 100, 256]
    wgs = [2, 4, 8, 8, 3, 4, 0]
    As, bs = _systems(14, sizes)
    A1, L0 = spd_inputs.integer_spd(400, seed=31)
    j = 250
    A1[j, j] -= L0[j, j] ** 2
    As[4] = A1
    nb = [_nb_single(n) for n in sizes]
    info, Ls, Xs = _run(tc, As, bs, nb, align=align, wgs=wgs)
    assert list(info) == [0, 0, 0, 0, j + 1, 0, 0]
    for s in (0, 1, 2, 3, 5, 6):
        Lo = oracle.cholesky(As[s])
        assert oracle.factor_error(Ls[s], Lo) <= TOL
        Xo = oracle.potrs(Lo, bs[s])
        assert np.max(np.abs(Xs[s] - Xo)) / np.max(np.abs(Xo)) <= TOL


@pytest.mark.parametrize("nrhs", [4, 1, 6])
def test_batched_one_tile_compact(tc, nrhs):
    """Every system one tile with even leading dimensions: the compact kernel
    instance (128-row slabs, two workgroups per compute unit).  Up to four
    right-hand sides ride along the factorization as its forward solve; six
    take the separate forward-solve task."""
    sizes = [1, 16, 17, 100, 128, 129, 200, 255, 256, 257, 300, 384, 385, 450, 511, 512]
    As, bs = _systems(21, sizes, nrhs)
    nb = [_nb_single(n) for n in sizes]
    info, Ls, Xs = _run(tc, As, bs, nb)
    assert np.all(info == 0)
    for A, b, L, X in zip(As, bs, Ls, Xs):
        Lo = oracle.cholesky(A)
        assert oracle.factor_error(L, Lo) <= TOL
        Xo = oracle.potrs(Lo, b)
        assert np.max(np.abs(X - Xo)) / max(np.max(np.abs(Xo)), 1e-300) <= TOL
        assert np.all(oracle.solve_backward_error(A, X, b) <= 1e-15)


def test_batched_one_tile_compact_bitwise_across_policies(tc):
    """The compact instance gives the same bits under every claim order, with
    the fused forward solve (four right-hand sides) and without (five)."""
    sizes = [400, 37, 512, 128, 250, 300, 16, 511]
    nb = [_nb_single(n) for n in sizes]
    for nrhs in (4, 5):
        As, bs = _systems(23, sizes, nrhs)
        ref = _run(tc, As, bs, nb)
        assert np.all(ref[0] == 0)
        for pol, seed in [(tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0), (tc.POLICY_RANDOM, 9)]:
            got = _run(tc, As, bs, nb, policy=pol, seed=seed)
            assert np.array_equal(got[0], ref[0])
            assert all(np.array_equal(a, b) for a, b in zip(got[1], ref[1]))
            assert all(np.array_equal(a, b) for a, b in zip(got[2], ref[2]))


def test_batched_one_tile_compact_integer_exact(tc):
    """Integer systems through the compact instance and its fused forward
    solve: L and X exact."""
    sizes = [64, 300, 17, 512, 129, 200, 1, 33]
    As, bs, L0s, X0s = [], [], [], []
    for i, n in enumerate(sizes):
        A, L0 = spd_inputs.integer_spd(n, seed=60 + i)
        b, x0 = spd_inputs.integer_rhs(A, 3, seed=60 + i)
        As.append(A), bs.append(b), L0s.append(L0), X0s.append(x0)
    info, Ls, Xs = _run(tc, As, bs, [_nb_single(n) for n in sizes])
    assert np.all(info == 0)
    for L, L0, X, X0 in zip(Ls, L0s, Xs, X0s):
        assert np.array_equal(L, L0)
        assert np.array_equal(X, X0)


def test_batched_integer_systems_exact(tc):
    sizes = [64, 300, 17, 512]
    As, bs, L0s, X0s = [], [], [], []
    for i, n in enumerate(sizes):
        A, L0 = spd_inputs.integer_spd(n, seed=40 + i)
        b, x0 = spd_inputs.integer_rhs(A, 3, seed=40 + i)
        As.append(A), bs.append(b), L0s.append(L0), X0s.append(x0)
    nb = [16, 128, 16, 512]
    info, Ls, Xs = _run(tc, As, bs, nb)
    assert np.all(info == 0)
    for L, L0, X, X0 in zip(Ls, L0s, Xs, X0s):
        assert np.array_equal(L, L0)
        assert np.array_equal(X, X0)


def test_batched_bitwise_across_policies(tc):
    sizes = [400, 37, 600, 128, 250]
    As, bs = _systems(13, sizes)
    nb = [_nb_single(400), 16, 128, 128, 64]
    ref = _run(tc, As, bs, nb)
    for pol, seed in [(tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0), (tc.POLICY_RANDOM, 5)]:
        got = _run(tc, As, bs, nb, policy=pol, seed=seed)
        assert np.array_equal(got[0], ref[0])
        assert all(np.array_equal(a, b) for a, b in zip(got[1], ref[1]))
        assert all(np.array_equal(a, b) for a, b in zip(got[2], ref[2]))


def test_batched_factor_only_and_empty(tc):
    As, bs = _systems(14, [100, 0, 50], nrhs=0)
    nb = [112, 16, 64]
    info, Ls, _ = _run(tc, As, bs, nb)
    assert np.all(info == 0)
    for A, L in zip(As, Ls):
        if A.shape[0]:
            assert oracle.factor_error(L, oracle.cholesky(A)) <= TOL
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert len(tc.factor_solve_batched_(e, [], [], e, [], [], [], 4)) == 0


def test_batched_config5_full_size(tc):
    """The timed batched launch at its full size: 4096 systems of orders
    uniform in [16, 512] (seed 4), 4 right-hand sides, tile sizes from the
    tuned table (the compact instance), one launch.  Every system: info 0,
    the scaled backward error of its factor ||A - L L^T||_F / (n eps ||A||_F)
    at most 10 and the normwise backward error of its solutions at most
    1e-13, both computed on the device in FP64 as checkers; 32 sampled
    systems (the smallest and largest among them) against the oracle to
    1e-10, with the oracle's long-double backward error at most 1e-15."""
    from paper_1402_6601_amd import autotune
    print("case: 4096 systems, seed 4, 4 RHS, tuned table", flush=True)
    ns, A0, a_off, lda, B0, b_off = spd_inputs.batched_systems_device(4096, 4, 4)
    nb = autotune.tile_sizes(ns)
    wgs = autotune.potrf_wgs(ns)
    A, B = A0.clone(), B0.clone()
    info = tc.factor_solve_batched_(A, a_off, lda, B, b_off, ns, nb, 4, wgs=wgs)
    torch.cuda.synchronize()
    assert np.all(info == 0)
    eps = np.finfo(np.float64).eps
    worst_beta, worst_eta = 0.0, 0.0
    for s_, (n, o, l, ob) in enumerate(zip(ns, a_off, lda, b_off)):
        n, o, l, ob = int(n), int(o), int(l), int(ob)
        S = A0[o:o + n * l].view(n, l)[:, :n]            # symmetric: row c = column c
        L = torch.tril(A[o:o + n * l].view(n, l)[:, :n].t())
        beta = float(torch.linalg.norm(S - L @ L.t().contiguous()) / (n * eps * torch.linalg.norm(S)))
        b = B0[ob:ob + n * 4].view(4, n).t()
        x = B[ob:ob + n * 4].view(4, n).t()
        r = b - S @ x.contiguous()
        an = float(torch.max(torch.sum(torch.abs(S), dim=1)))
        eta = torch.max(torch.abs(r), dim=0).values / (an * torch.max(torch.abs(x), dim=0).values +
                                                      torch.max(torch.abs(b), dim=0).values)
        worst_beta = max(worst_beta, beta)
        worst_eta = max(worst_eta, float(torch.max(eta)))
    print("worst beta %.3f, worst eta %.3e" % (worst_beta, worst_eta), flush=True)
    assert worst_beta <= 10.0
    assert worst_eta <= 1e-13
    rng = np.random.default_rng(5)
    sample = set(rng.choice(len(ns), size=30, replace=False).tolist()) | {int(np.argmin(ns)), int(np.argmax(ns))}
    for s_ in sorted(sample):
        n, o, l, ob = int(ns[s_]), int(a_off[s_]), int(lda[s_]), int(b_off[s_])
        Ah = A0[o:o + n * l].view(n, l)[:, :n].cpu().numpy()
        bh = B0[ob:ob + n * 4].view(4, n).t().cpu().numpy()
        Lh = np.tril(A[o:o + n * l].view(n, l)[:, :n].cpu().numpy().T)
        Xh = B[ob:ob + n * 4].view(4, n).t().cpu().numpy()
        Lo = oracle.cholesky(Ah)
        assert oracle.factor_error(Lh, Lo) <= TOL
        Xo = oracle.potrs(Lo, bh)
        assert np.max(np.abs(Xh - Xo)) / np.max(np.abs(Xo)) <= TOL
        assert np.all(oracle.solve_backward_error(Ah, Xh, bh) <= 1e-15)
