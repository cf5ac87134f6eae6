"""Priority-policy ablation of the factorization on one GPU.

    python -m paper_1402_6601_amd.policy_ablation [--n 32768] [--nb 512] [--reps 5] [--inv-trsm]

The persistent kernel's workers claim work items in a ticket order fixed
by the host planner.  Four orders are compared:

* rank   -- decreasing upward rank, the priority rule of HEFT that the
            paper's scheduler recalls (section 3.1); ties by (step, kind, i, j);
* fifo   -- step-major order (k ascending, then kind, i, j): the order a
            sequential tile algorithm issues its tasks in;
* random -- a random topological order (seeded).
* list   -- HEFT's list schedule: the work items in the order a simulation
            of 256 identical workers, each taking the ready item of highest
            upward rank, starts them.

Every order is topological, so all four compute the same tile operations
in the same per-tile order; the factor must be bitwise identical and only
the time may differ.  Prints one JSON line per policy and a summary line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--random-seeds", type=int, nargs="*", default=[1, 2])
    ap.add_argument("--inv-trsm", action="store_true",
                    help="the benchmark's factorization DAG: TRSMs through the diagonal tiles' inverses")
    args = ap.parse_args(argv)

    import numpy as np
    import torch
    import paper_1402_6601_amd as tc
    import spd_inputs

    tc.load()
    if not torch.cuda.is_available():
        print("policy_ablation needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    n, nb = args.n, args.nb
    A0, _ = spd_inputs.spd_matrix_device(n, args.seed, 1.0, device=dev)
    W = torch.empty_like(A0)
    ws = torch.empty(tc.workspace_bytes(tc.OP_FACTOR, n, nb), dtype=torch.uint8, device=dev)
    runs = [("rank", tc.POLICY_RANK, 0), ("list", tc.POLICY_LIST, 0), ("fifo", tc.POLICY_FIFO, 0)]
    runs += [("random", tc.POLICY_RANDOM, s) for s in args.random_seeds]
    ref = None
    results = []
    for name, pol, seed in runs:
        t_plan = time.perf_counter()
        tc.plan_query(tc.OP_FACTOR, n, nb, pol, seed)   # builds the plan outside the timed runs (inv_trsm: the warm-up)
        t_plan = time.perf_counter() - t_plan
        times = []
        for _ in range(args.reps + 1):                  # the first run is a warm-up
            W.copy_(A0)
            torch.cuda.synchronize()
            info, ms = tc.factor_(W, nb, policy=pol, seed=seed, ws=ws, want_kernel_ms=True, inv_trsm=args.inv_trsm)
            if info != 0:
                raise RuntimeError("factorization failed: info=%d" % info)
            times.append(ms)
        times = times[1:]
        L = torch.tril(W.mT)
        if ref is None:
            ref = L.clone()
            same = True
        else:
            same = bool(torch.equal(L, ref))
        mean = float(np.mean(times))
        rec = {"policy": name, "seed": seed, "n": n, "nb": nb, "reps": args.reps, "inv_trsm": args.inv_trsm,
               "kernel_ms_mean": round(mean, 3), "kernel_ms_min": round(float(np.min(times)), 3),
               "kernel_ms_max": round(float(np.max(times)), 3),
               "tflops": round(n ** 3 / 3.0 / (mean * 1e-3) / 1e12, 3),
               "plan_ms": round(t_plan * 1e3, 1), "bitwise_equal_to_rank": same}
        results.append(rec)
        print(json.dumps(rec), flush=True)
    base = results[0]["kernel_ms_mean"]
    print(json.dumps({"summary": {r["policy"] + ("" if r["policy"] != "random" else str(r["seed"])):
                                  round(r["kernel_ms_mean"] / base, 4) for r in results},
                      "all_bitwise_equal": all(r["bitwise_equal_to_rank"] for r in results)}), flush=True)
    return 0 if all(r["bitwise_equal_to_rank"] for r in results) else 3


if __name__ == "__main__":
    sys.exit(main())
