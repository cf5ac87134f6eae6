"""Autotuner of the batched launch: per order bucket, the tile size and the
workgroups that share a system's factorization.

    python -m paper_1402_6601_amd.autotune [--count 4096] [--seed 4] [--out tune_batched.json]

In a batched launch each system gets its own tile size nb.  One tile
(nb >= n) keeps a system's factorization on one workgroup, or, with wgs > 1
(orders above 128), on wgs workgroups that share the tile's sub-block DAG
(the split POTRF of the large factorizations); smaller tiles split its
factorization and solve into a DAG whose tasks spread over many workgroups.
Both shorten a system's critical path at the price of more, smaller work
items.  Which is faster depends on the order and on the rest of the batch,
so the tuner measures it, in the spirit of the history-based calibration of
the paper's performance model (section 2.3): the systems are grouped into
order buckets, and for every bucket each candidate (tile rule, wgs) is timed
on the GPU with a batch of that bucket's systems (kernel time from HIP
events, best of a few runs).  The fastest candidate per bucket goes into a
JSON table, which :func:`tile_sizes` and :func:`potrf_wgs` apply.  The table
finally is validated on the whole batch against the one-tile,
one-workgroup default, and both times are recorded in it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_batched.json")
BUCKETS = [(1, 64), (65, 128), (129, 192), (193, 256), (257, 320), (321, 384), (385, 448), (449, 512)]
# (tile rule, wgs): rule 0 is one tile per system; wgs > 1 shares a one-tile
# factorization above order 128 among that many workgroups
CANDIDATES = [(0, 1), (0, 2), (0, 4), (0, 8), (256, 0), (128, 0), (64, 0), (32, 0)]


def single_tile(n: int) -> int:
    return int(max(16, min(512, -(-int(n) // 16) * 16)))


def rule_nb(n: int, rule: int) -> int:
    """Tile size of a system of order n under a bucket rule (0 = one tile)."""
    if rule == 0 or rule >= n:
        return single_tile(n)
    return int(rule)


def load_table(path: str = DEFAULT_TABLE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _bucket_of(n, table):
    """(rule, wgs) of the table's bucket holding order n; (0, 0) if none.
    Entries are [lo, hi, rule] or [lo, hi, rule, wgs]."""
    if table:
        for e in table["buckets"]:
            if int(e[0]) <= n <= int(e[1]):
                return int(e[2]), (int(e[3]) if len(e) > 3 else 0)
    return 0, 0


def tile_sizes(ns, table=None):
    """Per-system tile sizes: the table's rule for each system's order bucket,
    one tile per system where no table (or bucket) applies."""
    if table is None:
        table = load_table()
    return np.asarray([rule_nb(int(n), _bucket_of(int(n), table)[0]) for n in ns], dtype=np.int32)


def potrf_wgs(ns, table=None):
    """Per-system workgroups sharing a one-tile factorization (tchol_opts.wgs):
    the bucket's choice for a system kept in one tile above order 128, else 0
    (one workgroup, or the default split of a tiled system)."""
    if table is None:
        table = load_table()
    out = []
    for n in ns:
        rule, w = _bucket_of(int(n), table)
        one_tile = rule_nb(int(n), rule) >= n
        out.append(w if (one_tile and n > 128 and w > 1) else 0)
    return np.asarray(out, dtype=np.int32)


def _time_batch(tc, torch, ns, A0, a_off, lda, B0, b_off, nb, nrhs, reps, ws=None, wgs=None):
    A = torch.empty_like(A0)
    B = torch.empty_like(B0)
    best = None
    for _ in range(reps):
        A.copy_(A0)
        B.copy_(B0)
        torch.cuda.synchronize()
        info, ms = tc.factor_solve_batched_(A, a_off, lda, B, b_off, ns, nb, nrhs, ws=ws, want_kernel_ms=True,
                                            wgs=wgs)
        if np.any(info != 0):
            raise RuntimeError("a system failed during tuning")
        best = ms if best is None else min(best, ms)
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    args = ap.parse_args(argv)

    import torch
    import paper_1402_6601_amd as tc
    import spd_inputs

    tc.load()
    if not torch.cuda.is_available():
        print("the autotuner needs a GPU", file=sys.stderr)
        return 1
    ns, A0, a_off, lda, B0, b_off = spd_inputs.batched_systems_device(args.count, args.seed, args.nrhs)
    print("[tune] %d systems generated" % len(ns), file=sys.stderr, flush=True)
    rules = []
    report = []
    for lo, hi in BUCKETS:
        idx = np.where((ns >= lo) & (ns <= hi))[0]
        if len(idx) == 0:
            continue
        sub = lambda arr: np.asarray(arr)[idx]
        times = {}
        for rule, w in CANDIDATES:
            if rule and rule >= hi:
                continue
            if w > 1 and hi <= 128:
                continue
            cand = {"buckets": [[lo, hi, rule, w]]}
            nb = tile_sizes(ns[idx], cand)
            wg = potrf_wgs(ns[idx], cand)
            times[(rule, w)] = _time_batch(tc, torch, sub(ns), A0, sub(a_off), sub(lda), B0, sub(b_off), nb,
                                           args.nrhs, args.reps, wgs=wg)
            print("[tune] bucket %d-%d (%d systems) nb rule %s, wgs %d: %.3f ms"
                  % (lo, hi, len(idx), rule or "one tile", w, times[(rule, w)]), file=sys.stderr, flush=True)
        best = min(times, key=times.get)
        rules.append([lo, hi, int(best[0]), int(best[1])])
        name = lambda c: ("one tile" if c[0] == 0 else "nb %d" % c[0]) + (", wgs %d" % c[1] if c[1] > 1 else "")
        report.append({"bucket": [lo, hi], "systems": int(len(idx)),
                       "ms": {name(c): round(t, 4) for c, t in times.items()}, "chosen": name(best)})
    table = {"device": torch.cuda.get_device_name(0), "count": args.count, "seed": args.seed, "nrhs": args.nrhs,
             "buckets": rules, "report": report}
    nb_tuned, wgs_tuned = tile_sizes(ns, table), potrf_wgs(ns, table)
    nb_default = np.array([single_tile(n) for n in ns], dtype=np.int32)
    t_tuned = _time_batch(tc, torch, ns, A0, a_off, lda, B0, b_off, nb_tuned, args.nrhs, args.reps, wgs=wgs_tuned)
    t_default = _time_batch(tc, torch, ns, A0, a_off, lda, B0, b_off, nb_default, args.nrhs, args.reps)
    table["validation_ms"] = {"tuned": round(t_tuned, 4), "one_tile_per_system": round(t_default, 4)}
    if t_default < t_tuned:
        # the per-bucket optimum did not carry over to the whole batch
        table["buckets"] = [[lo, hi, 0, 0] for lo, hi, _, _ in rules]
        table["validation_ms"]["kept"] = "one tile per system"
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({"table": args.out, "buckets": table["buckets"], "validation_ms": table["validation_ms"]}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
