"""Benchmark: tiled FP64 Cholesky factorization + 16-RHS solve on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One step is one pass of the whole hot path on one synthetic input: the
factorization A = L L^T and the tiled solve of 16 right-hand sides, run as
one merged tile DAG in one launch of the persistent kernel.  The workload is the FP64 case n = 32768,
nb = 512, A = B B^T / n + I with B uniform on [-1, 1] (seed 1), 16 RHS
uniform on [-1, 1].  Every timed step factors its own pristine copy of A
(all copies are made before the timed region; 288 GB of HBM holds them), so
no restore copy is timed.

Prints one JSON line: value = n^3/3 flops per step / step time (the solve's
flops are not counted), the roofline of that launch (n^3/3 flops / its mean
duration, measured with HIP events on its stream, against the 78.6 TFLOP/s
FP64 matrix peak), and the CPU oracle timed on the leading
principal block of the same matrix (whose factor is the leading block of L,
so it doubles as a parity check of that block).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Cholesky TFLOP/s (n^3/3), FP64 vs mixed+refined at 1e-12 residual, n=32768"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def device_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("tchol_device.hip", "kargs.h", "tchol_kinds.h"):
        with open(os.path.join(ROOT, "paper_1402_6601_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def ci95(xs):
    """Mean and the half-width of its 95 % confidence interval (Student t)."""
    if not xs:
        return None
    a = np.asarray(xs, dtype=np.float64)
    half = 0.0
    if len(a) > 1:
        from scipy import stats
        half = float(stats.t.ppf(0.975, len(a) - 1) * a.std(ddof=1) / np.sqrt(len(a)))
    return {"reps": len(a), "mean": round(float(a.mean()), 3), "ci95_half_width": round(half, 3),
            "min": round(float(a.min()), 3), "max": round(float(a.max()), 3)}


def load_traffic(n, nb):
    """Per-launch HBM bytes of the merged factor + solve launch from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source."""
    path = os.path.join(ROOT, "profiles", "traffic_factor_solve_n%d_nb%d.json" % (n, nb))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("device_source_sha256_16") != device_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def sampled_reconstruction(torch, W, A0, n, count=64, seed=123):
    """max |(L L^T)_ij - A_ij| / (n eps max|A|) over sampled (i, j), i >= j, with
    the sums in long double on the host.  W holds L in its column-major lower
    triangle (row-major column i of W = row i of L); A0 is the pristine input."""
    rng = np.random.default_rng(seed)
    amax = float(A0.abs().max().item())
    worst = 0.0
    for _ in range(count):
        i = int(rng.integers(0, n))
        j = int(rng.integers(0, i + 1))
        li = W[: i + 1, i].cpu().numpy().astype(np.longdouble)
        lj = W[: j + 1, j].cpu().numpy().astype(np.longdouble)
        s = np.sum(li[: j + 1] * lj[: j + 1])
        aij = float(A0[j, i].item())  # column-major (i, j) of the input
        worst = max(worst, abs(float(s) - aij))
    return worst / (n * 2.0 ** -52 * amax)


def sampled_solve_eta(torch, A0, B0, Xc, n, count=64, seed=321):
    """Normwise backward error of each right-hand side's solution over sampled
    rows of the residual b - A x, with the sums in long double on the host.
    B0: (n, nrhs) row-major right-hand sides; Xc: (nrhs, n), the solutions in
    column-major order; A0 the pristine symmetric input."""
    rng = np.random.default_rng(seed)
    rows = rng.choice(n, min(count, n), replace=False)
    Ar = A0[torch.as_tensor(rows, device=A0.device)].cpu().numpy().astype(np.longdouble)
    Xh = Xc.t().cpu().numpy()
    Bh = B0.cpu().numpy()
    R = Bh[rows].astype(np.longdouble) - Ar @ Xh.astype(np.longdouble)
    anorm = float(A0.abs().sum(dim=1).max().item())
    den = anorm * np.max(np.abs(Xh), axis=0) + np.max(np.abs(Bh), axis=0)
    return [float(v) for v in np.max(np.abs(R).astype(np.float64), axis=0) / den]


def cpu_model() -> str:
    """The host CPU's model name (Linux), for the record beside the oracle timings."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_small_config(oracle, reps=30):
    """The oracle on the small FP64 workload (n = 1024, seed 0, shift 1): factor
    plus one-RHS solve, `reps` runs on all host threads (mean and 95 % interval)
    and one run on a single thread."""
    import spd_inputs
    A, b = spd_inputs.spd_matrix_and_rhs(1024, 0, nrhs=1)
    def once():
        t = time.perf_counter()
        F, info = oracle.potrf(A)
        oracle.potrs(F, b)
        return (time.perf_counter() - t) * 1e3
    once()
    ms_all = [once() for _ in range(reps)]
    nthr = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        ms_one = once()
    finally:
        oracle.set_num_threads(nthr)
    return {"workload": "n=1024 factor + 1-RHS solve (seed 0)", "threads": nthr, "ms_all_threads": ci95(ms_all),
            "ms_one_thread": round(ms_one, 3)}


def run_calib_copy(nbytes: int, reps: int):
    """A plain elementwise copy kernel (b = a * 1) that reads and writes
    nbytes each, to scale the PMC byte counters (a same-dtype copy_ may be
    served by a DMA engine that the counters do not see)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n * 8, "reps": reps}), flush=True)


def run_batched(args):
    """4096 SPD systems, n_i uniform on [16, 512] (seed 4), A_i = B_i B_i^T / n_i + I,
    factor + 4-RHS solve of all of them in one launch per step, tile sizes from
    the autotuner's table (one tile per system where there is none)."""
    import torch
    import paper_1402_6601_amd as tc
    from paper_1402_6601_amd import autotune
    import spd_inputs

    tc.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    seed = 4 if args.seed == 1 else args.seed
    nrhs = 4
    K, Wm = args.steps, args.warmup
    fp32 = args.dtype == "f32"
    t0 = time.time()
    if fp32:
        # FP32 storage: lda = n + 3 rounded up to 4, systems 16-byte aligned
        ns, A0, a_off, lda, B0, b_off = spd_inputs.batched_systems_device(args.count, seed, nrhs, device=dev,
                                                                          align=4, pad=3, fp32=True)
    else:
        ns, A0, a_off, lda, B0, b_off = spd_inputs.batched_systems_device(args.count, seed, nrhs, device=dev)
    run = tc.factor_solve_batched_f32_ if fp32 else tc.factor_solve_batched_
    table = autotune.load_table()
    nb = autotune.tile_sizes(ns, table)
    # the FP32 launch factors each one-tile system on one workgroup
    wgs = None if fp32 else autotune.potrf_wgs(ns, table)
    extra = {} if fp32 else {"wgs": wgs}
    torch.cuda.synchronize()
    log("batched inputs ready in %.1f s (%d systems, sum n = %d)" % (time.time() - t0, len(ns), int(ns.sum())))
    wsb = tc.batched_f32_workspace_bytes(ns, nb, nrhs) if fp32 else tc.batched_workspace_bytes(ns, nb)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    As = [torch.empty_like(A0) for _ in range(K)]
    Bs = [torch.empty_like(B0) for _ in range(K)]
    Aw, Bw = torch.empty_like(A0), torch.empty_like(B0)
    for w in range(Wm):
        Aw.copy_(A0)
        Bw.copy_(B0)
        info = run(Aw, a_off, lda, Bw, b_off, ns, nb, nrhs, ws=ws, **extra)
        if np.any(info != 0):
            raise RuntimeError("batched factorization failed")
        log("warmup %d done" % (w + 1))
    for s_ in range(K):
        As[s_].copy_(A0)
        Bs[s_].copy_(B0)
    torch.cuda.synchronize()
    kernel_ms = []
    failed = []
    t_start = time.perf_counter()
    for s_ in range(K):
        info, ms = run(As[s_], a_off, lda, Bs[s_], b_off, ns, nb, nrhs, ws=ws, want_kernel_ms=True, **extra)
        kernel_ms.append(ms)
        if np.any(info != 0):   # the info array is read back by the call itself (host memory)
            failed.append(s_)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    if failed:
        raise RuntimeError("batched factorization failed in timed steps %s" % failed)
    ms_per_step = (t_end - t_start) * 1e3 / K
    kmean = float(np.mean(kernel_ms))
    n64 = ns.astype(np.float64)
    flops = float(np.sum(n64 ** 3) / 3.0)
    # algorithmic bytes: read the lower triangle of A, write L, read L in each
    # of the two substitutions, read and write the right-hand sides twice
    elem = 4.0 if fp32 else 8.0
    tri = float(np.sum(n64 * (n64 + 1) / 2.0)) * elem
    bytes_alg = 4.0 * tri + 4.0 * float(np.sum(n64)) * nrhs * elem
    achieved = bytes_alg / (kmean * 1e-3) / 1e9

    # checks on a sample of systems, and the oracle timed on the host on it
    import oracle
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(len(ns), size=min(64, len(ns)), replace=False))
    Ah0 = A0.cpu().numpy().astype(np.float64)
    Bh0 = B0.cpu().numpy().astype(np.float64)
    Ah = As[K - 1].cpu().numpy().astype(np.float64)
    Bh = Bs[K - 1].cpu().numpy().astype(np.float64)
    worst_l, worst_x, worst_beta = 0.0, 0.0, 0.0
    tcpu = 0.0
    for i in sample:
        n_, o, l, ob = int(ns[i]), int(a_off[i]), int(lda[i]), int(b_off[i])
        Ai = np.ascontiguousarray(Ah0[o:o + n_ * l].reshape(n_, l)[:, :n_])
        bi = np.ascontiguousarray(Bh0[ob:ob + n_ * nrhs].reshape(nrhs, n_).T)
        Lg = np.tril(Ah[o:o + n_ * l].reshape(n_, l)[:, :n_].T)
        Xg = Bh[ob:ob + n_ * nrhs].reshape(nrhs, n_).T
        tc0 = time.perf_counter()
        F, inf = oracle.potrf(Ai)
        Xo = oracle.potrs(F, bi)
        tcpu += time.perf_counter() - tc0
        worst_l = max(worst_l, oracle.factor_error(Lg, F))
        worst_x = max(worst_x, float(np.max(np.abs(Xg - Xo)) / np.max(np.abs(Xo))))
        if fp32:
            S_ = oracle.sym_from_lower(Ai)
            worst_beta = max(worst_beta, float(np.linalg.norm(S_ - Lg @ Lg.T) /
                                               (n_ * 2.0 ** -23 * np.linalg.norm(S_))))
    sample_flops = float(np.sum(n64[sample] ** 3) / 3.0)
    out = {
        "metric": "Cholesky TFLOP/s (sum of n_i^3/3), batched factor + 4-RHS solve in one launch"
                  + (", FP32 storage" if fp32 else ""),
        "value": round(flops / (ms_per_step * 1e-3) / 1e12, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": "batched %s factor + solve, %d systems, n_i ~ U{16..512} (seed %d), "
                               "A_i = B_i B_i^T/n_i + I, 4 RHS, one persistent launch"
                               % ("fp32 (fp32 updates, fp64 diagonal tiles and solves)" if fp32 else "fp64",
                                  len(ns), seed),
                   "count": int(len(ns)), "seed": seed, "nrhs": nrhs,
                   "tile_table": "tuned" if table else "one tile per system",
                   "systems_split_into_tiles": int(np.sum(nb < ns)),
                   "systems_on_several_workgroups": 0 if fp32 else int(np.sum(wgs > 1))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "tchol_persistent (batched factor + solve DAG)", "kernel_ms_mean": round(kmean, 3),
                     "bytes_per_launch": bytes_alg, "flops_per_launch": flops,
                     "mfma_frac": round(flops / (kmean * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4)},
        "kernel_ms": [round(x, 3) for x in kernel_ms],
        "e_L_max_sampled": worst_l,
        "e_x_max_sampled": worst_x,
        "beta32_max_sampled": worst_beta if fp32 else None,
        "cpu_baseline": {"value": round(sample_flops / tcpu / 1e12, 6), "unit": "TFLOP/s",
                         "cores": oracle.num_threads(), "kind": "oracle",
                         "sample": "oracle FP64 factor + solve of %d sampled systems of the same batch "
                                   "(factor flops only counted); %.3f s" % (len(sample), tcpu)},
    }
    print(json.dumps(out), flush=True)

FP32_MFMA_PEAK_TFLOPS = 157.3


BF16_MFMA_PEAK_TFLOPS = 2500.0


def measure_mixed(torch, tc, dev, n, nb, nrhs, seed, shift, K, Wm, policy, fp64_ms=None, tol=1e-12, maxit=30,
                  lowp=None):
    """Mixed-precision solve with refinement to eta <= tol of nrhs right-hand
    sides of A = B B^T / n + shift I (B ~ U[-1, 1], seed), timed per step
    (factor + refinement, A resident; every step starts from the original
    right-hand sides).  fp64_ms: FP64 factor + solve time of the same order
    to compare against; None measures it here on the same matrix.  Returns
    a dict of the results."""
    import spd_inputs
    lowp = tc.LOWP_FP32 if lowp is None else lowp
    bf16 = lowp == tc.LOWP_BF16
    t0 = time.time()
    A, rng = spd_inputs.spd_matrix_device(n, seed, shift, device=dev)
    B0 = torch.from_numpy(spd_inputs.rhs(rng, n, nrhs)).to(dev)
    B0c = B0.t().contiguous()
    torch.cuda.synchronize()
    log("mixed (%s updates): inputs ready in %.1f s (n=%d nb=%d nrhs=%d shift=%g seed=%d)"
        % ("bf16" if bf16 else "fp32", time.time() - t0, n, nb, nrhs, shift, seed))
    ws = torch.empty(tc.mixed_workspace_bytes(n, nb, nrhs, lowp), dtype=torch.uint8, device=dev)
    X = torch.empty_like(B0c)
    for w in range(Wm):
        X.copy_(B0c)
        rc, it, berr = tc.solve_mixed_(A, X, nb, tol=tol, maxit=maxit, policy=policy, ws=ws, lowp=lowp)
        log("mixed warmup %d: rc=%d iterations=%d max eta=%.3g" % (w + 1, rc, it, float(np.max(berr))))
    steps = []
    for s_ in range(K):
        X.copy_(B0c)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        rc, it, berr, fms = tc.solve_mixed_(A, X, nb, tol=tol, maxit=maxit, policy=policy, ws=ws,
                                             want_kernel_ms=True, lowp=lowp)
        torch.cuda.synchronize()
        steps.append(((time.perf_counter() - ts) * 1e3, rc, it, float(np.max(berr)), fms))
        log("mixed step %d: %.3f ms rc=%d iterations=%d max eta=%.3g factor kernel %.3f ms"
            % (s_ + 1, steps[-1][0], rc, it, steps[-1][3], fms))
    if any(st[1] != 0 for st in steps):
        raise RuntimeError("mixed solve did not converge: %s" % [st[1] for st in steps])
    ms = float(np.mean([st[0] for st in steps]))
    fms = float(np.mean([st[4] for st in steps]))
    # independent check of the last solution: FP64 residual with torch's product
    # (whole matrix), and 64 sampled rows with long-double sums on the host
    R = B0 - A @ X.t()
    anorm = float(A.abs().sum(dim=1).max().item())
    eta_full = (R.abs().amax(dim=0) / (anorm * X.t().abs().amax(dim=0) + B0.abs().amax(dim=0))).cpu().numpy()
    rng_s = np.random.default_rng(7)
    Xh = X.t().cpu().numpy().astype(np.longdouble)
    Bh = B0.cpu().numpy()
    worst_row = 0.0
    for i in rng_s.integers(0, n, size=64):
        row = A[int(i)].cpu().numpy().astype(np.longdouble)
        r = Bh[int(i)] - row @ Xh
        worst_row = max(worst_row, float(np.max(np.abs(r))))
    out = {"ms_per_solve": round(ms, 3), "factor_kernel_ms": round(fms, 3),
           "refinement_iterations": [st[2] for st in steps], "eta_reported_max": max(st[3] for st in steps),
           "eta_check_max": float(np.max(eta_full)), "abs_residual_sampled_rows_max": worst_row,
           "value": round(n ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3), "tol": tol}
    peak = BF16_MFMA_PEAK_TFLOPS if bf16 else FP32_MFMA_PEAK_TFLOPS
    out["lowp"] = "bf16" if bf16 else "fp32"
    out["factor_roofline"] = {"bound": "mfma", "achieved": round(n ** 3 / 3.0 / (fms * 1e-3) / 1e12, 3),
                              "peak": peak, "unit": "TFLOP/s",
                              "frac": round(n ** 3 / 3.0 / (fms * 1e-3) / 1e12 / peak, 4),
                              "note": ("GEMM updates on BF16 matrix cores (three BF16 terms per operand, six term "
                                       "products, FP32 accumulation); SYRK FP32; POTRF and TRSM in FP64; achieved "
                                       "counts n^3/3, not the six BF16 products" if bf16 else
                                       "trailing updates on FP32 matrix cores; POTRF and TRSM in FP64")}
    del ws
    if fp64_ms is None:
        # the FP64 path of the benchmark: factorization and solve in one launch
        ws_m = torch.empty(tc.factor_solve_workspace_bytes(n, nb, nrhs), dtype=torch.uint8, device=dev)
        Wt = torch.empty_like(A)
        t64 = []
        for s_ in range(max(1, K)):
            Wt.copy_(A)
            X.copy_(B0c)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            if tc.factor_solve_(Wt, X, nb, policy=policy, ws=ws_m) != 0:
                raise RuntimeError("fp64 factorization failed")
            torch.cuda.synchronize()
            t64.append((time.perf_counter() - ts) * 1e3)
        fp64_ms = float(np.mean(t64))
        R = B0 - A @ X.t()
        out["fp64_eta_max"] = float((R.abs().amax(dim=0) / (anorm * X.t().abs().amax(dim=0) +
                                                           B0.abs().amax(dim=0))).max().item())
        out["fp64_measured_on"] = "the same matrix (merged factor + solve launch)"
        del Wt, ws_m
    else:
        out["fp64_measured_on"] = "the fp64 workload's matrix of the same order (its time does not depend on values)"
    out["fp64_ms_per_solve"] = round(fp64_ms, 3)
    out["speedup_vs_fp64"] = round(fp64_ms / ms, 3)
    del A, X
    torch.cuda.empty_cache()
    return out


def run_mixed(args):
    """The mixed-precision workload alone: n = 32768, nb = 512, A = B B^T/n + 1e-4 I
    (seed 2), 16 right-hand sides refined to eta <= 1e-12, against FP64 on the
    same matrix."""
    import torch
    import paper_1402_6601_amd as tc
    tc.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed = 2 if args.seed == 1 else args.seed
    policy = {"rank": tc.POLICY_RANK, "fifo": tc.POLICY_FIFO, "random": tc.POLICY_RANDOM, "list": tc.POLICY_LIST}[args.policy]
    lowp = tc.LOWP_BF16 if args.lowp == "bf16" else tc.LOWP_FP32
    r = measure_mixed(torch, tc, dev, args.n, args.nb, args.nrhs, seed, 1e-4, args.steps, args.warmup, policy,
                      lowp=lowp)
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("bf16+f32+f64" if args.lowp == "bf16" else "f32+f64"),
        "data": "synthetic",
        "config": {"workload": "mixed %s/fp64 Cholesky + iterative refinement of %d RHS to eta<=1e-12, "
                               "n=%d, nb=%d, A=B*B^T/n+1e-4*I, B~U[-1,1] (seed %d)"
                               % (args.lowp, args.nrhs, args.n, args.nb, seed),
                   "n": args.n, "nb": args.nb, "nrhs": args.nrhs, "seed": seed, "shift": 1e-4},
        "roofline": r["factor_roofline"],
        "mixed": r,
    }
    print(json.dumps(out), flush=True)


def measure_adjoint(torch, tc, dev, n, nb, seed, K, Wm, policy, cpu_sample_n=0):
    """The adjoint of the factorization (tchol_backward) of A = B B^T / n + I
    (B ~ U[-1, 1], seed) for an upstream Lbar = tril(N(0, 1)) drawn after B.
    Timed per call with every step starting from the original Lbar (copies
    made beforehand).  Nominal flops (2/3) n^3: the two GEMM updates of each
    reversed step.  Check at full size: the bilinear identity
    <Abar, E> = <Lbar, dL> for a random symmetric E, with
    dL = L Phi(L^{-1} E L^{-T}) from torch's triangular solves."""
    import spd_inputs
    t0 = time.time()
    A, rng = spd_inputs.spd_matrix_device(n, seed, 1.0, device=dev)
    Lbar = torch.from_numpy(spd_inputs.lower_upstream(rng, n)).to(dev)
    W = A.clone()
    if tc.factor_(W, nb, policy=policy) != 0:
        raise RuntimeError("factorization failed")
    Gb0 = Lbar.mT.contiguous()                 # column-major lower = Lbar
    torch.cuda.synchronize()
    log("adjoint: inputs ready in %.1f s (n=%d nb=%d seed=%d)" % (time.time() - t0, n, nb, seed))
    ws = torch.empty(tc.workspace_bytes(tc.OP_BACKWARD, n, nb), dtype=torch.uint8, device=dev)
    G = torch.empty_like(Gb0)
    for w in range(Wm):
        G.copy_(Gb0)
        tc.backward_(W, G, nb, policy=policy, ws=ws)
    Gs = [Gb0.clone() for _ in range(K)]
    torch.cuda.synchronize()
    kms = []
    ts = time.perf_counter()
    for s_ in range(K):
        _, ms = tc.backward_(W, Gs[s_], nb, policy=policy, ws=ws, want_kernel_ms=True)
        kms.append(ms)
    torch.cuda.synchronize()
    ms_call = (time.perf_counter() - ts) * 1e3 / K
    kmean = float(np.mean(kms))
    flops = 2.0 * n ** 3 / 3.0
    # check: <Abar, E> against <Lbar, L Phi(L^{-1} E L^{-T})>
    L = torch.tril(W.mT)
    low = torch.tril(Gs[-1].mT)
    Abar = low + torch.tril(low, -1).mT
    gen = torch.Generator(device=dev)
    gen.manual_seed(17)
    E = torch.randn(n, n, dtype=torch.float64, device=dev, generator=gen)
    E = E + E.mT
    X = torch.linalg.solve_triangular(L, E, upper=False)          # L^{-1} E
    Y = torch.linalg.solve_triangular(L, X.mT, upper=False).mT    # L^{-1} E L^{-T}
    Phi = torch.tril(Y) - 0.5 * torch.diag_embed(torch.diagonal(Y))
    dL = L @ Phi
    lhs = float((Abar * E).sum().item())
    rhs = float((torch.tril(Lbar) * dL).sum().item())
    out = {"ms_per_call": round(ms_call, 3), "kernel_ms_mean": round(kmean, 3),
           "kernel_ms": [round(x, 3) for x in kms],
           "value": round(flops / (ms_call * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "flops_nominal": flops,
           "bilinear_check_rel": abs(lhs - rhs) / max(abs(rhs), 1e-300)}
    out["roofline"] = {"bound": "mfma", "achieved": round(flops / (kmean * 1e-3) / 1e12, 3),
                       "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(flops / (kmean * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
                       "kernel": "tchol_persistent (reverse factorization DAG)"}
    if cpu_sample_n > 0:
        import oracle
        m = min(cpu_sample_n, n)
        Ah, rs = spd_inputs.spd_matrix(m, seed)
        Lh = oracle.cholesky(Ah)
        Lbh = spd_inputs.lower_upstream(rs, m)
        tcpu = time.perf_counter()
        oracle.chol_adjoint(Lh, Lbh)
        tcpu = time.perf_counter() - tcpu
        out["cpu_baseline"] = {"value": round(2.0 * m ** 3 / 3.0 / tcpu / 1e12, 6), "unit": "TFLOP/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "oracle adjoint (reverse of the unblocked factorization) at n=%d of the "
                                         "same matrix family; %.2f s" % (m, tcpu)}
    del A, W, Gs, G, ws
    torch.cuda.empty_cache()
    return out


def run_adjoint(args):
    """The adjoint workload alone: n = 8192, nb = 256, A = B B^T/n + I (seed 3)."""
    import torch
    import paper_1402_6601_amd as tc
    tc.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed = 3 if args.seed == 1 else args.seed
    n = 8192 if args.n == 32768 else args.n
    nb = 256 if args.nb == 512 else args.nb
    policy = {"rank": tc.POLICY_RANK, "fifo": tc.POLICY_FIFO, "random": tc.POLICY_RANDOM, "list": tc.POLICY_LIST}[args.policy]
    r = measure_adjoint(torch, tc, dev, n, nb, seed, args.steps, args.warmup, policy,
                        cpu_sample_n=min(args.cpu_sample_n, 3072))
    out = {
        "metric": "Cholesky adjoint TFLOP/s ((2/3) n^3 nominal), n=%d" % n,
        "value": r["value"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_call"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fp64 blocked Cholesky adjoint, n=%d, nb=%d, A=B*B^T/n+I, B~U[-1,1] (seed %d), "
                               "Lbar=tril(N(0,1))" % (n, nb, seed), "n": n, "nb": nb, "seed": seed},
        "roofline": r["roofline"],
        "adjoint": r,
    }
    if "cpu_baseline" in r:
        out["cpu_baseline"] = r["cpu_baseline"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ci-reps", type=int, default=30,
                    help="factor workload: extra launches (restored in between) for the mean and its 95%% interval")
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--policy", choices=["rank", "fifo", "random", "list"], default="list")
    ap.add_argument("--cpu-sample-n", type=int, default=8192,
                    help="order of the leading block the CPU oracle factors (0 = skip)")
    ap.add_argument("--calib-copy", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--workload", choices=["factor", "batched", "mixed", "adjoint"], default="factor",
                    help="factor: the n=32768 factor + solve (default); batched: 4096 systems in one launch; "
                         "mixed: the mixed-precision solve with refinement alone")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="factor workload: skip the adjoint measurement appended to the line")
    ap.add_argument("--no-mixed", action="store_true",
                    help="factor workload: skip the mixed-precision comparison appended to the line")
    ap.add_argument("--count", type=int, default=4096, help="batched: number of systems")
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64", help="batched: storage precision")
    ap.add_argument("--lowp", choices=["bf16", "fp32"], default="bf16",
                    help="mixed: precision of the trailing GEMM updates")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build runs the factorization on a single MI355X "
              "(--gpus %d requested); multi-GPU sharding is a design note only." % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        run_calib_copy(args.calib_copy, max(1, args.steps))
        return
    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "mixed":
        run_mixed(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return

    import torch
    import paper_1402_6601_amd as tc
    import spd_inputs

    tc.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n, nb, nrhs, K, Wm = args.n, args.nb, args.nrhs, args.steps, args.warmup
    policy = {"rank": tc.POLICY_RANK, "fifo": tc.POLICY_FIFO, "random": tc.POLICY_RANDOM, "list": tc.POLICY_LIST}[args.policy]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.time()
    A0, rng = spd_inputs.spd_matrix_device(n, args.seed, 1.0, device=dev)
    B0 = torch.from_numpy(spd_inputs.rhs(rng, n, nrhs)).to(dev)      # (n, nrhs) row-major
    B0c = B0.t().contiguous()                                          # column-major copy
    torch.cuda.synchronize()
    log("inputs ready in %.1f s (n=%d nb=%d nrhs=%d)" % (time.time() - t0, n, nb, nrhs))

    ws_f = torch.empty(tc.workspace_bytes(tc.OP_FACTOR, n, nb), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(tc.workspace_bytes(tc.OP_SOLVE, n, nb, nrhs), dtype=torch.uint8, device=dev)
    ws_fs = torch.empty(tc.load().tchol_factor_solve_workspace_bytes(n, nb, nrhs), dtype=torch.uint8, device=dev)
    work = [torch.empty_like(A0) for _ in range(K)]
    rhs = [torch.empty_like(B0c) for _ in range(K)]
    stream = torch.cuda.current_stream(dev)

    def step(Wt, Bt, kernel_ms):
        # one launch: the factorization and the solve as one merged DAG
        info, ms = tc.factor_solve_(Wt, Bt, nb, policy=policy, ws=ws_fs, want_kernel_ms=True)
        if info != 0:
            raise RuntimeError("factorization failed: info=%d" % info)
        kernel_ms.append(ms)

    # warmup: reuse the first working copy, restoring it (untimed) every time
    for w in range(Wm):
        work[0].copy_(A0)
        rhs[0].copy_(B0c)
        step(work[0], rhs[0], [])
        log("warmup %d done" % (w + 1))
    for s in range(K):
        work[s].copy_(A0)
        rhs[s].copy_(B0c)
    torch.cuda.synchronize()

    kernel_ms = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record(stream)
    for s in range(K):
        step(work[s], rhs[s], kernel_ms)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / K
    log("timed %d steps: %.3f ms/step (events %.3f ms/step), factor + solve kernel mean %.3f ms"
        % (K, ms_per_step, ev0.elapsed_time(ev1) / K, float(np.mean(kernel_ms))))

    # checks on the result of the last timed step (before any later launch):
    # sampled entries of L L^T and sampled rows of its solve's residual, both
    # in long double; the leading block of its L is kept for the oracle
    recon = sampled_reconstruction(torch, work[K - 1], A0, n)
    eta_rows = sampled_solve_eta(torch, A0, B0, rhs[K - 1], n)
    m_lead = min(args.cpu_sample_n, n) if args.cpu_sample_n > 0 else 0
    L_lead = np.tril(work[K - 1][:m_lead, :m_lead].cpu().numpy().T) if m_lead else None
    log("last timed step: sampled reconstruction %.3e (bound 10), sampled solve eta %.3e"
        % (recon, max(eta_rows)))
    if not recon <= 10.0:
        raise RuntimeError("sampled reconstruction error %.3e exceeds the backward-error bound 10" % recon)
    if not max(eta_rows) <= 1e-14:
        raise RuntimeError("sampled solve backward error %.3e above FP64 level" % max(eta_rows))

    flops = n ** 3 / 3.0
    value = flops / (ms_per_step * 1e-3) / 1e12
    kmean = float(np.mean(kernel_ms))
    achieved = flops / (kmean * 1e-3) / 1e12
    traffic = load_traffic(n, nb)

    # for the record: the factorization and the solve as two launches
    Wt = work[0]
    Wt.copy_(A0)
    # the factorization alone, with the merged launch's TRSMs (through the inverses)
    _, factor_alone_ms = tc.factor_(Wt, nb, policy=policy, ws=ws_f, want_kernel_ms=True, inv_trsm=True)
    Bt = rhs[0]
    Bt.copy_(B0c)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    _, solve_kernel_ms = tc.solve_(Wt, Bt, nb, ws=ws_s, want_kernel_ms=True)
    solve_ms = (time.perf_counter() - ts) * 1e3

    # repeated launches for a confidence interval: A and B restored (untimed)
    # before each one, the kernel timed by HIP events on the launch stream
    rep_ms = []
    for r in range(args.ci_reps):
        work[0].copy_(A0)
        rhs[0].copy_(B0c)
        step(work[0], rhs[0], rep_ms)
    torch.cuda.synchronize()
    if args.ci_reps:
        log("repeated %d launches: kernel mean %.3f ms" % (args.ci_reps, float(np.mean(rep_ms))))

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fp64 tiled Cholesky factor + %d-RHS solve, n=%d, nb=%d, A=B*B^T/n+I, B~U[-1,1] "
                               "(seed %d)" % (nrhs, n, nb, args.seed),
                   "n": n, "nb": nb, "nrhs": nrhs, "seed": args.seed, "policy": args.policy},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
                     "traffic": traffic, "kernel": "tchol_persistent (merged factorization + solve DAG)",
                     "kernel_ms_mean": round(kmean, 3), "flops_per_launch": flops,
                     "flops_note": "n^3/3; the solve's 4 n^2 nrhs flops in the same launch are not counted"},
        "step_kernel_ms": [round(x, 3) for x in kernel_ms],
        "kernel_ms_repeated": ci95(rep_ms),
        "factor_alone_kernel_ms": round(factor_alone_ms, 3),
        "factor_alone_frac": round(flops / (factor_alone_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
        "solve_ms": round(solve_ms, 3),
        "solve_kernel_ms": round(solve_kernel_ms, 3),
        "solve_hbm_gbs": round(n * n * 8.0 / (solve_kernel_ms * 1e-3) / 1e9, 1),
        "reconstruction_err_sampled": recon,
        "solve_eta_sampled_max": max(eta_rows),
    }
    del work, rhs

    if not args.no_mixed:
        # the mixed-precision solve of the same order (its own matrix family: shift 1e-4,
        # seed 2), compared with this run's FP64 factor + solve time
        del ws_s
        torch.cuda.empty_cache()
        out["mixed_refined"] = measure_mixed(torch, tc, dev, n, nb, nrhs, 2, 1e-4, 2, 1, policy,
                                             fp64_ms=ms_per_step, lowp=tc.LOWP_BF16)
        out["mixed_refined_fp32"] = measure_mixed(torch, tc, dev, n, nb, nrhs, 2, 1e-4, 2, 1, policy,
                                                  fp64_ms=ms_per_step, lowp=tc.LOWP_FP32)
        ws_s = None

    if not args.no_adjoint:
        # the adjoint workload (n = 8192, nb = 256, seed 3), summarised on the same line
        out["adjoint"] = measure_adjoint(torch, tc, dev, 8192, 256, 3, 3, 1, policy)

    if args.cpu_sample_n > 0:
        import oracle
        m = min(args.cpu_sample_n, n)
        lead = A0[:m, :m].cpu().numpy()          # row-major buffer = column-major A (symmetric)
        Ahost = np.ascontiguousarray(lead.T)      # logical matrix read by the library
        log("oracle: factoring the leading %d x %d block on %d threads" % (m, m, oracle.num_threads()))
        tcpu = time.perf_counter()
        F, info = oracle.potrf(Ahost)
        tcpu = time.perf_counter() - tcpu
        Lg = L_lead   # the leading block of the last timed step's L
        out["cpu_baseline"] = {"value": round((m ** 3 / 3.0) / tcpu / 1e12, 6), "unit": "TFLOP/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "oracle FP64 unblocked Cholesky of the leading %dx%d principal block of "
                                         "the same n=%d matrix (its factor is the leading block of L); %.2f s"
                                         % (m, m, n, tcpu),
                               "seconds": round(tcpu, 3), "cpu_model": cpu_model(),
                               "small_config": oracle_small_config(oracle)}
        out["e_L_leading_block"] = oracle.factor_error(Lg, F) if info == 0 else None
        if out["e_L_leading_block"] is None or not out["e_L_leading_block"] <= 1e-10:
            raise RuntimeError("leading block of L disagrees with the oracle: %s" % out["e_L_leading_block"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
