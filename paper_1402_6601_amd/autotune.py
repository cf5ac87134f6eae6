"""Autotuner of the batched launch's tile sizes.

    python -m paper_1402_6601_amd.autotune [--count 4096] [--seed 4] [--out tune_batched.json]

In a batched launch each system gets its own tile size nb.  One tile
(nb >= n) keeps a system on a single workgroup; smaller tiles split its
factorization and solve into a DAG whose tasks spread over many
workgroups, which shortens that system's critical path at the price of more
tasks.  Which is faster depends on the order and on the rest of the batch,
so the tuner measures it: the systems are grouped into order buckets, and
for every bucket each candidate tile size is timed on the GPU with a batch
of that bucket's systems (kernel time from HIP events, best of a few runs).
The fastest candidate per bucket goes into a JSON table, which
:func:`tile_sizes` applies.  The table finally is validated on the whole
batch against the one-tile-per-system default, and both times are recorded
in it.
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
CANDIDATES = [0, 256, 128, 64, 32]   # 0: one tile per system


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


def tile_sizes(ns, table=None):
    """Per-system tile sizes: the table's rule for each system's order bucket,
    one tile per system where no table (or bucket) applies."""
    if table is None:
        table = load_table()
    rules = []
    if table:
        rules = [(int(lo), int(hi), int(r)) for lo, hi, r in table["buckets"]]
    out = []
    for n in ns:
        r = 0
        for lo, hi, rr in rules:
            if lo <= n <= hi:
                r = rr
                break
        out.append(rule_nb(int(n), r))
    return np.asarray(out, dtype=np.int32)


def _time_batch(tc, torch, ns, A0, a_off, lda, B0, b_off, nb, nrhs, reps, ws=None):
    A = torch.empty_like(A0)
    B = torch.empty_like(B0)
    best = None
    for _ in range(reps):
        A.copy_(A0)
        B.copy_(B0)
        torch.cuda.synchronize()
        info, ms = tc.factor_solve_batched_(A, a_off, lda, B, b_off, ns, nb, nrhs, ws=ws, want_kernel_ms=True)
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
        for cand in CANDIDATES:
            if cand and cand >= hi:
                continue
            nb = np.array([rule_nb(int(n), cand) for n in ns[idx]], dtype=np.int32)
            times[cand] = _time_batch(tc, torch, sub(ns), A0, sub(a_off), sub(lda), B0, sub(b_off), nb, args.nrhs,
                                      args.reps)
            print("[tune] bucket %d-%d (%d systems) nb rule %s: %.3f ms" % (lo, hi, len(idx), cand or "one tile",
                                                                          times[cand]), file=sys.stderr, flush=True)
        best = min(times, key=times.get)
        rules.append([lo, hi, int(best)])
        report.append({"bucket": [lo, hi], "systems": int(len(idx)),
                       "ms": {("one tile" if c == 0 else str(c)): round(t, 4) for c, t in times.items()},
                       "chosen": "one tile" if best == 0 else int(best)})
    table = {"device": torch.cuda.get_device_name(0), "count": args.count, "seed": args.seed, "nrhs": args.nrhs,
             "buckets": rules, "report": report}
    nb_tuned = tile_sizes(ns, table)
    nb_default = np.array([single_tile(n) for n in ns], dtype=np.int32)
    t_tuned = _time_batch(tc, torch, ns, A0, a_off, lda, B0, b_off, nb_tuned, args.nrhs, args.reps)
    t_default = _time_batch(tc, torch, ns, A0, a_off, lda, B0, b_off, nb_default, args.nrhs, args.reps)
    table["validation_ms"] = {"tuned": round(t_tuned, 4), "one_tile_per_system": round(t_default, 4)}
    if t_default < t_tuned:
        # the per-bucket optimum did not carry over to the whole batch
        table["buckets"] = [[lo, hi, 0] for lo, hi, _ in rules]
        table["validation_ms"]["kept"] = "one tile per system"
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({"table": args.out, "buckets": table["buckets"], "validation_ms": table["validation_ms"]}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
