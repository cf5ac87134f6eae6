"""Per-kind work-item timing of one launch, from the kernel's trace buffer.

    python -m paper_1402_6601_amd.trace_report [--op factor|merged|mixed|solve|adjoint|batched] [--n N] [--nb NB]
        [--policy P]

The persistent kernel can record, per work item, the wall clock (100 MHz)
when its ticket was claimed, when its wait ended, when it finished, and the
task and workgroup (``tchol_opts.trace``).  This tool runs one launch of the
chosen DAG on a synthetic input of the benchmark family (factor: shift 1,
seed 1; merged: the same factorization and its 16-RHS solve as one
launch; mixed: shift 1e-4, seed 2, the factorization launch of the
mixed-precision solve; solve: the 16-RHS forward and backward solve launch
on the factor of the seed-1 matrix; adjoint: shift 1, seed 3,
Lbar = tril N(0, 1); batched: 4096 systems of orders uniform in [16, 512],
seed 4, factor and 4-RHS solve in one launch, tiles from the tuned table), and
prints the makespan, the fraction of worker time spent running and waiting,
per task kind the item count and mean / median / max duration and mean wait,
and the busy fraction over time in 20 buckets.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def report(tc, plan, trace, tag, out=print):
    tr = trace.cpu().numpy().reshape(-1, 4).astype(np.int64)
    claim, start, end, tw = tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3]
    task = tw & 0xffffffff
    wg = tw >> 32
    kind = plan["kind"][task]
    t0 = claim.min()
    span = (end.max() - t0) / 100.0
    busy = (end - start) / 100.0
    wait = (start - claim) / 100.0
    nwg = len(np.unique(wg))
    out("[%s] makespan %.2f ms, workgroups %d, busy %.3f, waiting %.3f"
        % (tag, span / 1000, nwg, busy.sum() / (nwg * span), wait.sum() / (nwg * span)))
    out("  %-6s %8s %10s %10s %10s %11s %10s" % ("kind", "items", "mean us", "p50 us", "max us", "sum ms", "wait us"))
    for k in range(len(tc.KIND_NAMES)):
        m = kind == k
        if m.any():
            out("  %-6s %8d %10.1f %10.1f %10.1f %11.1f %10.1f" % (
                tc.KIND_NAMES[k], m.sum(), busy[m].mean(), np.median(busy[m]), busy[m].max(), busy[m].sum() / 1000,
                wait[m].mean()))
    # tasks split into several work items (the POTRF pools): the task's span,
    # from its first item's start to its last item's end
    for k in range(len(tc.KIND_NAMES)):
        m = kind == k
        if not m.any() or len(np.unique(task[m])) == m.sum():
            continue
        ids, inv = np.unique(task[m], return_inverse=True)
        t_first = np.full(len(ids), np.iinfo(np.int64).max)
        t_last = np.zeros(len(ids), dtype=np.int64)
        np.minimum.at(t_first, inv, start[m])
        np.maximum.at(t_last, inv, end[m])
        sp = (t_last - t_first) / 100.0
        if tc.KIND_NAMES[k] == "POTRF":
            out("  %-6s task span: mean %.1f us, p50 %.1f us, max %.1f us over %d tasks, sum %.2f ms"
                % (tc.KIND_NAMES[k], sp.mean(), np.median(sp), sp.max(), len(ids), sp.sum() / 1000))
    edges = np.linspace(0, span, 21)
    s_rel, e_rel = (start - t0) / 100.0, (end - t0) / 100.0
    util = []
    for b in range(20):
        ov = np.clip(np.minimum(e_rel, edges[b + 1]) - np.maximum(s_rel, edges[b]), 0, None)
        util.append(ov.sum() / (nwg * (edges[b + 1] - edges[b])))
    out("  busy over time: " + " ".join("%.2f" % u for u in util))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", choices=["factor", "merged", "mixed", "solve", "adjoint", "batched"], default="factor")
    ap.add_argument("--count", type=int, default=4096, help="batched: number of systems")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--policy", choices=["rank", "list", "fifo", "random"], default="list")
    ap.add_argument("--lowp", choices=["bf16", "fp32"], default="bf16", help="mixed: precision of the GEMM updates")
    args = ap.parse_args(argv)
    import torch
    import paper_1402_6601_amd as tc
    import spd_inputs
    tc.load()
    if not torch.cuda.is_available():
        print("trace_report needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    pol = {"rank": tc.POLICY_RANK, "list": tc.POLICY_LIST, "fifo": tc.POLICY_FIFO, "random": tc.POLICY_RANDOM}[args.policy]
    if args.op == "batched":
        # 4096 systems of orders uniform in [16, 512] (seed 4), 4 right-hand
        # sides each, tile sizes from the tuned table: factor + solve in one launch
        from paper_1402_6601_amd import autotune
        ns, A0, a_off, lda, B0, b_off = spd_inputs.batched_systems_device(args.count, 4, 4)
        # --nb: that tile size for every system larger than it instead of the table
        nbs = (autotune.tile_sizes(ns) if not args.nb else
               np.array([autotune.rule_nb(int(x), args.nb) for x in ns], dtype=np.int32))
        wgs = autotune.potrf_wgs(ns) if not args.nb else None
        plan = tc.batched_plan_query(ns, nbs, pol, wgs=wgs)
        trace = torch.zeros(4 * plan["nitem"], dtype=torch.int64, device=dev)
        A, B = A0.clone(), B0.clone()
        tc.factor_solve_batched_(A, a_off, lda, B, b_off, ns, nbs, 4, policy=pol, wgs=wgs)
        A.copy_(A0)
        B.copy_(B0)
        _, ms = tc.factor_solve_batched_(A, a_off, lda, B, b_off, ns, nbs, 4, policy=pol, want_kernel_ms=True,
                                         trace=trace, wgs=wgs)
        print("kernel %.3f ms (HIP events), %d systems, sum n = %d" % (ms, len(ns), int(ns.sum())), flush=True)
        report(tc, plan, trace, args.op)
        return 0
    if args.op == "adjoint":
        n, nb = args.n or 8192, args.nb or 256
        A, rng = spd_inputs.spd_matrix_device(n, 3, 1.0, device=dev)
        Lb = torch.from_numpy(spd_inputs.lower_upstream(rng, n)).to(dev).mT.contiguous()
        W = A.clone()
        tc.factor_(W, nb)
        plan = tc.plan_query(tc.OP_BACKWARD, n, nb, pol)
        trace = torch.zeros(4 * plan["nitem"], dtype=torch.int64, device=dev)
        G = Lb.clone()
        tc.backward_(W, G, nb, policy=pol)
        G.copy_(Lb)
        _, ms = tc.backward_(W, G, nb, policy=pol, want_kernel_ms=True, trace=trace)
    else:
        n, nb = args.n or 32768, args.nb or 512
        mixed = args.op == "mixed"
        A, rng = spd_inputs.spd_matrix_device(n, 2 if mixed else 1, 1e-4 if mixed else 1.0, device=dev)
        # the mixed-precision factorization's DAG also holds the TRTRI tasks
        plan = tc.plan_query(tc.OP_MIXED_FACTOR if mixed else tc.OP_FACTOR, n, nb, pol)
        trace = torch.zeros(4 * plan["nitem"], dtype=torch.int64, device=dev)
        if mixed:
            B = torch.from_numpy(spd_inputs.rhs(rng, n, 16)).to(dev).t().contiguous()
            X = B.clone()
            lowp = tc.LOWP_BF16 if args.lowp == "bf16" else tc.LOWP_FP32
            tc.solve_mixed_(A, X, nb, maxit=0, policy=pol, lowp=lowp)
            X.copy_(B)
            _, _, _, ms = tc.solve_mixed_(A, X, nb, maxit=0, policy=pol, want_kernel_ms=True, trace=trace, lowp=lowp)
        elif args.op == "merged":
            # the benchmark's launch: factorization and 16-RHS solve as one DAG
            plan = tc.plan_query(tc.OP_FACTOR_SOLVE, n, nb, pol)
            trace = torch.zeros(4 * plan["nitem"], dtype=torch.int64, device=dev)
            B = torch.from_numpy(spd_inputs.rhs(rng, n, 16)).to(dev).t().contiguous()
            W, X = A.clone(), B.clone()
            tc.factor_solve_(W, X, nb, policy=pol)
            W.copy_(A)
            X.copy_(B)
            _, ms = tc.factor_solve_(W, X, nb, policy=pol, want_kernel_ms=True, trace=trace)
        elif args.op == "solve":
            plan = tc.plan_query(tc.OP_SOLVE, n, nb, pol)
            trace = torch.zeros(4 * plan["nitem"], dtype=torch.int64, device=dev)
            tc.factor_(A, nb, policy=pol)
            B = torch.from_numpy(spd_inputs.rhs(rng, n, 16)).to(dev).t().contiguous()
            X = B.clone()
            tc.solve_(A, X, nb, policy=pol)
            X.copy_(B)
            _, ms = tc.solve_(A, X, nb, policy=pol, want_kernel_ms=True, trace=trace)
        else:
            W = A.clone()
            tc.factor_(W, nb, policy=pol)
            W.copy_(A)
            _, ms = tc.factor_(W, nb, policy=pol, want_kernel_ms=True, trace=trace)
    print("kernel %.3f ms (HIP events), n=%d nb=%d" % (ms, n, nb), flush=True)
    report(tc, plan, trace, args.op)
    return 0


if __name__ == "__main__":
    sys.exit(main())
