"""Host planner of the batched launch: many systems' factor + solve DAGs merged
into one (no GPU).

Each system's tasks are checked against the same independent derivation as
the single-system plans: replaying its factorization and then its solve in
program order, with the tiles of the factor and the blocks of the
right-hand sides as the data (section 2, data-flow model), and keeping the
edges no path implies, must give exactly the planner's edges for that system,
and no edge may join two systems.  Claim orders must be topological and the
ranks must follow HEFT's recurrence (section 3.1) with the weights scaled to
a common flop unit, (nb / 16)^3 per system.
"""
import collections

import numpy as np
import pytest

from tests import tiled_ref

tc = pytest.importorskip("paper_1402_6601_amd")

POTRF, TRSM, SYRK, GEMM, FTRSV, FGEMV, BTRSV, BGEMV = range(8)
WEIGHT = {POTRF: 5, TRSM: 10, SYRK: 4, GEMM: 6, FTRSV: 1, FGEMV: 2, BTRSV: 1, BGEMV: 2, tiled_ref.GEMM2: 12}


def bplan(n, nb, policy=0, seed=0):
    try:
        return tc.batched_plan_query(n, nb, policy, seed)
    except ImportError as e:  # library not built
        pytest.skip(str(e))


def reduce_transitively(out, keep=lambda b: False):
    """Drop the edges (a, b) a longer path implies, except into tasks b that
    ``keep`` names (the factorization lists every panel a merged update
    reads, even when its chain already orders the two)."""
    succ = collections.defaultdict(set)
    for a, b in out:
        succ[a].add(b)

    def reachable(a, b):
        stack = [x for x in succ[a] if x != b]
        seen = set()
        while stack:
            x = stack.pop()
            if x == b:
                return True
            if x in seen:
                continue
            seen.add(x)
            stack.extend(succ[x])
        return False

    return {(a, b) for (a, b) in out if keep(b) or not reachable(a, b)}


def dataflow_edges_factor_solve(T, inv=(), tri=False):
    """Program-order replay of the tile factorization then the two tiled
    substitutions; edges join each access to the last writer of the datum
    (tiles ("L", i, j), right-hand-side blocks ("B", i); for the diagonal
    tiles in ``inv``, their inverses ("D", k) and the blocks ("S", k) of y).
    tri: the factorization's TRSMs apply the inverses of tiles 0 .. T-2."""
    last_writer = {}
    out = set()

    def access(task, reads, writes):
        for d in list(reads) + list(writes):
            if d in last_writer and last_writer[d] != task:
                out.add((last_writer[d], task))
        for d in writes:
            last_writer[d] = task

    tile = lambda d: d if isinstance(d[0], str) else ("L",) + d
    for task, reads, writes in tiled_ref.factor_program(T, tri):
        access(task, [tile(r) for r in reads], [tile(w) for w in writes])
    for task, reads, writes in tiled_ref.solve_program(T, inv, given=range(T - 1) if tri else ()):
        access(task, reads, writes)
    return reduce_transitively(out, keep=lambda b: b[0] in (POTRF, TRSM, SYRK, GEMM, tiled_ref.GEMM2))


def key(p, t):
    return (int(p["kind"][t]), int(p["i"][t]), int(p["j"][t]), int(p["k"][t]))


def system_edges(p):
    per = collections.defaultdict(set)
    for t in range(p["ntask"]):
        for e in range(p["succ_off"][t], p["succ_off"][t + 1]):
            s = int(p["succ"][e])
            assert p["sys"][t] == p["sys"][s], "an edge joins two systems"
            per[int(p["sys"][t])].add((key(p, t), key(p, s)))
    return per


SIZES = [
    ([16], [16]),
    ([100, 600, 0, 16], [512, 256, 16, 16]),
    ([48, 33, 64], [16, 16, 32]),
    ([1, 17, 200, 512, 513], [16, 16, 64, 128, 512]),
]


@pytest.mark.parametrize("n,nb", SIZES)
def test_batched_edges_equal_dataflow(n, nb):
    p = bplan(n, nb)
    per = system_edges(p)
    for s, (ns, nbs) in enumerate(zip(n, nb)):
        T = -(-ns // nbs)
        assert per.get(s, set()) == dataflow_edges_factor_solve(T), (s, ns, nbs)
        # every task of the system is present
        cnt = collections.Counter(int(k) for k, q in zip(p["kind"], p["sys"]) if q == s)
        npair = sum((T - 1 - j) * ((j - 1) // 2) for j in range(1, T))
        ng = T * (T - 1) * (T - 2) // 6 - 2 * npair
        assert cnt.get(POTRF, 0) == T == cnt.get(FTRSV, 0) == cnt.get(BTRSV, 0)
        assert cnt.get(TRSM, 0) == cnt.get(SYRK, 0) == T * (T - 1) // 2 == cnt.get(FGEMV, 0) == cnt.get(BGEMV, 0)
        assert cnt.get(GEMM, 0) == ng and cnt.get(tiled_ref.GEMM2, 0) == npair


@pytest.mark.parametrize("n,nb", [(16, 16), (100, 16), (1024, 128), (1000, 128), (200, 64)])
def test_factor_solve_plan_equals_dataflow(n, nb):
    """The merged factor + solve launch of one system: the explicit inverse of
    every diagonal tile whose order is a multiple of 16 (TRTRI(k) after
    POTRF(k)), applied by the factorization's TRSM(., k) for k < T - 1 and
    by the solve's row strips; a ragged last tile substitutes in place."""
    try:
        p = tc.plan_query(tc.OP_FACTOR_SOLVE, n, nb)
    except ImportError as e:  # library not built
        pytest.skip(str(e))
    T = -(-n // nb)
    inv = [k for k in range(T) if min(nb, n - k * nb) % 16 == 0]
    got = {(key(p, t), key(p, int(p["succ"][e])))
           for t in range(p["ntask"]) for e in range(p["succ_off"][t], p["succ_off"][t + 1])}
    assert got == dataflow_edges_factor_solve(T, inv, tri=True)
    # TRSM items are 128-row blocks of the inverse's product
    for t in range(p["ntask"]):
        if int(p["kind"][t]) == TRSM:
            assert p["parts"][t] == -(-min(nb, n - nb * int(p["i"][t])) // 128)
    w = dict(WEIGHT)
    w[tiled_ref.TRTRI] = 10
    for t in range(p["ntask"]):
        succ = [p["rank"][p["succ"][e]] for e in range(p["succ_off"][t], p["succ_off"][t + 1])]
        assert p["rank"][t] == w[int(p["kind"][t])] * (nb // 16) ** 3 + (max(succ) if succ else 0)


@pytest.mark.parametrize("policy,seed", [(tc.POLICY_LIST, 0), (tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0),
                                         (tc.POLICY_RANDOM, 3)])
def test_batched_claim_order_is_topological(policy, seed):
    n, nb = [1, 17, 200, 512, 513, 300], [16, 16, 64, 128, 512, 128]
    p = bplan(n, nb, policy, seed)
    nt = p["ntask"]
    first = {}
    for idx, t in enumerate(p["item_task"]):
        first.setdefault(int(t), idx)
    assert len(first) == nt
    for t in range(nt):
        for e in range(p["succ_off"][t], p["succ_off"][t + 1]):
            assert first[t] < first[int(p["succ"][e])]


def test_batched_ranks_follow_scaled_recurrence():
    n, nb = [64, 600, 300, 1000], [16, 256, 128, 512]
    p = bplan(n, nb, tc.POLICY_RANK)
    for t in range(p["ntask"]):
        u = nb[int(p["sys"][t])] // 16
        succ = [p["rank"][p["succ"][e]] for e in range(p["succ_off"][t], p["succ_off"][t + 1])]
        assert p["rank"][t] == WEIGHT[int(p["kind"][t])] * u ** 3 + (max(succ) if succ else 0)
    # decreasing rank along the claim order
    r = p["rank"][p["item_task"]]
    assert np.all(np.diff(r) <= 0)


def test_batched_plan_of_nothing():
    p = bplan([0, 0], [16, 16])
    assert p["ntask"] == 0 and p["nitem"] == 0


def test_batched_argument_checks():
    with pytest.raises(tc.TcholError):
        bplan([10, 20], [16, 24])          # nb not a multiple of 16
    with pytest.raises(tc.TcholError):
        bplan([10, -1], [16, 16])          # negative order
    assert tc.batched_workspace_bytes([100, 600], [512, 256]) > 0


def test_shared_factorization_parts():
    """wgs splits the POTRF of one-tile systems above 128 into that many work
    items (at most the sub-block pool's width), and changes nothing else:
    the same tasks, edges and claim order of tasks."""
    n = [100, 129, 300, 512, 512, 600]
    nb = [112, 144, 304, 512, 512, 256]
    wgs = [4, 2, 8, 3, 0, 8]
    p0 = bplan(n, nb)
    p1 = tc.batched_plan_query(n, nb, wgs=wgs)
    assert p1["ntask"] == p0["ntask"] and p1["nedge"] == p0["nedge"]
    assert np.array_equal(p1["kind"], p0["kind"]) and np.array_equal(p1["succ"], p0["succ"])
    POTRF = 0
    for t in range(p0["ntask"]):
        s, kind = int(p0["sys"][t]), int(p0["kind"][t])
        if kind != POTRF or nb[s] < n[s]:
            assert p1["parts"][t] == p0["parts"][t]
            continue
        assert p0["parts"][t] == 1
        want = 1 if (n[s] <= 128 or wgs[s] <= 1) else min(wgs[s], {129: 1, 300: 6, 512: 8}[n[s]])
        assert p1["parts"][t] == want
    assert p1["nitem"] == int(np.sum(p1["parts"]))
    # the workspace query covers any wgs choice: 8 bytes per work item
    assert tc.batched_workspace_bytes(n, nb) >= tc.batched_workspace_bytes([n[0], n[5]], [nb[0], nb[5]])
    with pytest.raises(tc.TcholError):
        tc.batched_plan_query(n, nb, wgs=[0, 0, 9, 0, 0, 0])


def test_tuned_table_rules():
    """tile_sizes / potrf_wgs apply a table's bucket rules: one tile (order
    rounded up to 16, at most 512), a fixed tile size below the order, and
    shared factorizations only for one-tile systems above 128."""
    from paper_1402_6601_amd import autotune
    table = {"buckets": [[1, 64, 0, 0], [65, 200, 0, 4], [201, 400, 128, 2], [401, 512, 0]]}
    ns = np.array([1, 16, 17, 64, 65, 128, 129, 200, 201, 255, 400, 401, 512])
    nb = autotune.tile_sizes(ns, table)
    assert list(nb) == [16, 16, 32, 64, 80, 128, 144, 208, 128, 128, 128, 416, 512]
    w = autotune.potrf_wgs(ns, table)
    assert list(w) == [0, 0, 0, 0, 0, 0, 4, 4, 0, 0, 0, 0, 0]
    # no table: one tile, one workgroup; orders outside every bucket likewise
    assert list(autotune.tile_sizes([40, 300], {"buckets": []})) == [48, 304]
    assert list(autotune.potrf_wgs([40, 300], {"buckets": []})) == [0, 0]
    assert list(autotune.tile_sizes([600], table)) == [512]
    # the committed table parses and covers every order of the workload
    t = autotune.load_table()
    if t is not None:
        orders = np.arange(16, 513)
        assert np.all(autotune.tile_sizes(orders, t) % 16 == 0)
        assert np.all(autotune.tile_sizes(orders, t) <= 512)
        assert np.all((autotune.potrf_wgs(orders, t) >= 0) & (autotune.potrf_wgs(orders, t) <= 8))
