"""Host planner of the adjoint's reverse tile DAG (no GPU).

The reverse program, per step k from T-1 down to 0,
    GREV(i, k, j)  Lbar_ik -= Q_ij L_jk      i > k, j = T-1 .. k+1 (links above
                   k+1 paired from the top into GREV2 tasks of two)
    TREV(i, k)     P_ik = Lbar_ik L_kk^{-1}   (writes Q_ik and Q_ki; through
                   L_kk^{-T} from TRTRI(k))
    DPART(i, k)    S_ik = tril(P_ik^T L_ik)
    DRED(k)        Lbar_kk -= sum_i S_ik     (k < T-1)
    PREV(k)        P_kk (writes Q_kk)
and, for a diagonal tile whose order is a multiple of 16, the closed form
in place of PREV(k):
    TRTRI(k)       L_kk^{-T}
    DRED(k)        also for k = T-1; leaves Lbar_kk^T in the Q_kk tile
    PADJM(k)       M = Phi(L_kk^T Lbar_kk)    (reads Lbar_kk^T)
    PADJY(k)       Y^T = (M L_kk^{-1})^T
    PADJS(k)       Q_kk = S, Lbar_kk = tril(S) / 2
is replayed in program order with its data (Lbar tiles, the P tile behind
each Q tile, the partial products S) and every read-after-write,
write-after-read and write-after-write conflict becomes an edge (section 2,
data-flow model).  The planner's edges must imply exactly the same order:
the two edge sets have equal transitive reductions.  Claim orders must be
topological, task counts as derived, and ranks must follow the upward-rank
recurrence (section 3.1).
"""
import collections

import numpy as np
import pytest

tc = pytest.importorskip("paper_1402_6601_amd")

GREV, TREV, DPART, PREV, TRTRI, DRED, PADJM, PADJY, PADJS, GREV2 = 8, 9, 10, 11, 12, 13, 15, 16, 17, 18
WEIGHT = {GREV: 6, TREV: 3, DPART: 3, PREV: 4, TRTRI: 40, DRED: 1, PADJM: 1, PADJY: 1, PADJS: 2, GREV2: 11}


def grev_tasks(k, T):
    """The chain into Lbar_ik as tasks (kind, js) in chain order: its last
    link j = k + 1 alone, the links above it paired from the top."""
    out, j = [], T - 1
    while j > k:
        if j - 1 >= k + 2 and (T - 1 - j) % 2 == 0:
            out.append((GREV2, (j, j - 1)))
            j -= 2
        else:
            out.append((GREV, (j,)))
            j -= 1
    return out
PRB = 64


def closed(m):
    """The diagonal tile of order m takes the closed-form adjoint."""
    return m % 16 == 0


def bplan(n, nb, policy=0, seed=0):
    try:
        return tc.plan_query(tc.OP_BACKWARD, n, nb, policy, seed)
    except ImportError as e:
        pytest.skip(str(e))


def reduce_transitively(edges):
    succ = collections.defaultdict(set)
    for a, b in edges:
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

    return {(a, b) for (a, b) in edges if not reachable(a, b)}


def dataflow_edges(n, nb):
    T = -(-n // nb)
    tsz = lambda t: min(nb, n - nb * t)
    last_writer, readers = {}, collections.defaultdict(set)
    out = set()

    def access(task, reads, writes):
        for d in reads:
            if d in last_writer and last_writer[d] != task:
                out.add((last_writer[d], task))
        for d in writes:
            if d in last_writer and last_writer[d] != task:
                out.add((last_writer[d], task))
            for r in readers[d]:
                if r != task:
                    out.add((r, task))
        for d in reads:
            readers[d].add(task)
        for d in writes:
            last_writer[d] = task
            readers[d] = set()

    def q(i, j):  # the P tile behind Q_ij
        return ("P", max(i, j), min(i, j))

    for k in range(T - 1, -1, -1):
        for i in range(k + 1, T):
            for kind, js in grev_tasks(k, T):
                access((kind, i, min(js), k), [q(i, j) for j in js] + [("Lbar", i, k)], [("Lbar", i, k)])
        if closed(tsz(k)):   # L_kk^{-T}, for TREV and the tile's adjoint
            access((TRTRI, k, k, k), [], [("IT", k)])
        for i in range(k + 1, T):
            access((TREV, i, k, k), [("Lbar", i, k), ("IT", k)], [("Lbar", i, k), ("P", i, k)])
        for i in range(k + 1, T):
            access((DPART, i, k, k), [("P", i, k)], [("S", i, k)])
        if closed(tsz(k)):
            # Lbar_kk^T goes into the storage of the P tile behind Q_kk
            access((DRED, k, k, k), [("S", i, k) for i in range(k + 1, T)] + [("Lbar", k, k)],
                   [("Lbar", k, k), ("P", k, k)])
            access((PADJM, k, k, k), [("P", k, k)], [("M", k)])
            access((PADJY, k, k, k), [("M", k), ("IT", k)], [("Y", k)])
            access((PADJS, k, k, k), [("Y", k), ("IT", k)], [("Lbar", k, k), ("P", k, k)])
        else:
            if k + 1 < T:
                access((DRED, k, k, k), [("S", i, k) for i in range(k + 1, T)] + [("Lbar", k, k)],
                       [("Lbar", k, k)])
            access((PREV, k, k, k), [("Lbar", k, k)], [("Lbar", k, k), ("P", k, k)])
    return reduce_transitively(out)


def key(p, t):
    return (int(p["kind"][t]), int(p["i"][t]), int(p["j"][t]), int(p["k"][t]))


@pytest.mark.parametrize("n,nb", [(16, 16), (40, 16), (100, 16), (130, 32), (512, 128), (1000, 256), (200, 160),
                                  (600, 256)])
def test_backward_edges_equal_dataflow(n, nb):
    p = bplan(n, nb)
    T = -(-n // nb)
    edges = set()
    for t in range(p["ntask"]):
        for e in range(p["succ_off"][t], p["succ_off"][t + 1]):
            edges.add((key(p, t), key(p, int(p["succ"][e]))))
    assert reduce_transitively(edges) == dataflow_edges(n, nb)
    cnt = collections.Counter(int(x) for x in p["kind"])
    ragged = int(not closed(n - nb * (T - 1)))   # only the last tile can be ragged
    assert cnt[PREV] == ragged and cnt[PADJM] == cnt[PADJY] == cnt[PADJS] == cnt[TRTRI] == T - ragged
    assert cnt[DRED] == T - ragged
    assert cnt[TREV] == cnt[DPART] == T * (T - 1) // 2
    assert cnt[GREV] + 2 * cnt[GREV2] == sum((T - k - 1) ** 2 for k in range(T))
    assert cnt[GREV] == sum((T - k - 1) * (1 + (T - k - 2) % 2) for k in range(T - 1))


@pytest.mark.parametrize("policy,seed", [(tc.POLICY_LIST, 0), (tc.POLICY_RANK, 0), (tc.POLICY_FIFO, 0),
                                         (tc.POLICY_RANDOM, 7)])
def test_backward_claim_order_is_topological(policy, seed):
    p = bplan(700, 128, policy, seed)
    first = {}
    for idx, t in enumerate(p["item_task"]):
        first.setdefault(int(t), idx)
    assert len(first) == p["ntask"]
    for t in range(p["ntask"]):
        for e in range(p["succ_off"][t], p["succ_off"][t + 1]):
            assert first[t] < first[int(p["succ"][e])]


def test_backward_ranks_and_parts():
    p = bplan(600, 256)
    for t in range(p["ntask"]):
        succ = [p["rank"][p["succ"][e]] for e in range(p["succ_off"][t], p["succ_off"][t + 1])]
        assert p["rank"][t] == WEIGHT[int(p["kind"][t])] + (max(succ) if succ else 0)
    tsz = lambda i: min(256, 600 - 256 * i)
    for t in range(p["ntask"]):
        kind, i, k = int(p["kind"][t]), int(p["i"][t]), int(p["k"][t])
        tri = lambda s: s * (s + 1) // 2
        want = {GREV: -(-tsz(i) // PRB) * -(-tsz(k) // PRB), GREV2: -(-tsz(i) // 128) * -(-tsz(k) // 128),
                TREV: -(-tsz(i) // PRB),
                DPART: tri(-(-tsz(k) // PRB)), PREV: 1, DRED: -(-tsz(k) // 16), TRTRI: -(-tsz(k) // 32),
                PADJM: tri(-(-tsz(k) // PRB)), PADJY: tri(-(-tsz(k) // PRB)), PADJS: tri(-(-tsz(k) // PRB))}[kind]
        assert p["parts"][t] == want
    # the inverses have no predecessors and a large weight: the first task
    # claimed is the inverse of the last diagonal tile that takes the closed
    # form (tile 1; the last tile, of order 88, is ragged)
    assert int(p["kind"][p["item_task"][0]]) == TRTRI and int(p["k"][p["item_task"][0]]) == 1


def test_backward_workspace_and_limits():
    b = tc.workspace_bytes(tc.OP_BACKWARD, 1000, 256)
    np_ = 1008
    assert b >= 2 * 8 * np_ * np_ + 8 * 6 * 256 * 256
    with pytest.raises(tc.TcholError):
        tc.workspace_bytes(tc.OP_BACKWARD, 16 * 200, 16)   # beyond the adjoint's tile count
