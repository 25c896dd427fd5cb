#!/usr/bin/env python3
"""Benchmark of direct TSQR on one MI355X.

A step is one pass of the whole hot path over one synthetic input already resident in HBM:
for the default workload (svd-c50: A = G diag(s) V^T, 4,000,000 x 50, s = logspace(0,-12,50))
one tsqr_svd call returning Q, R, U, S and V.  `value` is the whole-job rate in algorithmic GB/s:
A is read once and Q and U are written once (8 m n bytes each).

Prints ONE JSON line.  Extra fields: `roofline` for the dominant kernel (HIP events around each
launch, on the launch stream, over the timed region), `cpu_baseline` (the CPU oracle on a
bounded row sample of the same workload, on this host's cores), `accuracy` (the paper's success
metrics, Sec. I-B, computed with the oracle's long-double metric routines), `kernels`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3
FP64_RIDGE = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)

METRIC = "TSQR GB/s and % HBM roofline vs plain FP64; ||Q^T Q-I||, backward rel err"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="svd-c50",
                    choices=["svd-c50", "qr-small", "mixed-c25", "grad-c100", "batch512",
                             "batch512-f32"])
    ap.add_argument("--rows", type=int, default=0, help="override m (same recipe and seed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def level0_flops(m, n, b, form_q):
    """Householder QR of every b x n panel (2 b n^2 - 2/3 n^3) [+ explicit Q1, the same count]."""
    full, tail = divmod(m, b)
    per = lambda r: 2.0 * r * n * n - 2.0 / 3.0 * n ** 3 if r >= n else 2.0 * r * n * n
    f = full * per(b) + (per(tail) if tail else 0.0)
    return f * (2.0 if form_q else 1.0)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on exactly one GPU (--gpus 1); sharding the row blocks "
              "over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1301_1071_amd as tsqr
    from paper_1301_1071_amd import _lib
    import workloads

    dev = torch.device("cuda:0")
    name = args.workload
    if name.startswith("batch512"):
        return bench_batched(args, torch.float32 if name.endswith("f32") else torch.float64)
    cfg = workloads.CONFIGS[name]
    m = args.rows or cfg["m"]
    n = cfg["n"]
    A_h = workloads.config_matrix(name, m=m)
    A = torch.from_numpy(A_h).to(dev)
    torch.cuda.synchronize()

    if name == "svd-c50":
        U = torch.empty((m, n), dtype=torch.float64, device=dev)
        S = torch.empty((n,), dtype=torch.float64, device=dev)
        V = torch.empty((n, n), dtype=torch.float64, device=dev)
        Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(tsqr.workspace_bytes("svd", m, n), dtype=torch.uint8, device=dev)

        def step():
            tsqr.svd(A, want_qr=True, ws=ws, out=(U, S, V, Q, R), check_info=False)
        alg_bytes = 3 * 8.0 * m * n          # read A, write Q and U
        desc = "direct TSQR + SVD (Q, R, U, S, V), A = G diag(logspace(0,-12)) V^T"
        out_q = Q
        precision = "fp64"
    elif name == "grad-c100":
        # one differentiable pass: forward QR, then the QR adjoint for cotangents (dQ, dR)
        precision = "fp64"
        ct = workloads.cotangents(m, n)
        dQ = torch.from_numpy(ct["dQ"]).to(dev)
        dR = torch.from_numpy(ct["dR"]).to(dev)
        Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        dA = torch.empty((m, n), dtype=torch.float64, device=dev)
        ws = torch.empty(max(tsqr.workspace_bytes("qr", m, n),
                             tsqr.workspace_bytes("qr_backward", m, n)), dtype=torch.uint8,
                         device=dev)

        def step():
            tsqr.qr(A, ws=ws, out=(Q, R), check_info=False)
            tsqr.qr_backward(A, dQ, dR, ws=ws, out=dA, check_info=False)
        alg_bytes = 2 * 8.0 * m * n + 3 * 8.0 * m * n   # fwd: A, Q; bwd: A, dQ, dA
        desc = "direct TSQR forward (Q, R) + closed-form QR adjoint (dA), Q recomputed from A"
        out_q = Q
    else:
        precision = "fp64" if name == "qr-small" else "fp32_refined"
        Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(tsqr.workspace_bytes("qr", m, n, precision), dtype=torch.uint8, device=dev)

        def step():
            tsqr.qr(A, precision=precision, ws=ws, out=(Q, R), check_info=False)
        alg_bytes = 2 * 8.0 * m * n          # read A, write Q
        desc = "direct TSQR (Q, R)" + (" FP32 panels + FP64 refinement" if precision != "fp64" else "")
        out_q = Q

    if args.copy_probe:
        # a plain copy of known size (1 GiB read + 1 GiB written) to calibrate HBM counters
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.profile_collect()
    _lib.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.profile_enable(False)
    prof = _lib.profile_collect()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = alg_bytes / (ms_step * 1e-3) / 1e9

    # ---- per-kernel breakdown and the dominant kernel's roofline
    kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
               for k, v in prof.items() if v[1] > 0}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    dom_ms_launch = prof[dom][0] / prof[dom][1]
    plan_op = "svd" if name == "svd-c50" else "qr"
    roof = roofline(dom, dom_ms_launch, m, n, plan_op, precision, _lib)
    roof["kernel"] = dom
    roof["ms_per_launch"] = dom_ms_launch
    if args.rows == 0 and precision == "fp64":
        roof["traffic"] = MEASURED_TRAFFIC.get((name, dom))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": name, "m": m, "n": n, "desc": desc,
                   "seed": workloads.SEEDS[name], "algorithmic_bytes": alg_bytes},
        "hbm_frac": value / HBM_PEAK_GBS,
        "rows_per_s": m / (ms_step * 1e-3),
        "roofline": roof,
        "kernels": kernels,
    }

    if not args.no_accuracy:
        import oracle
        Qh = out_q.cpu().numpy()
        Rh = R.cpu().numpy()
        normA = oracle.norm2(A_h)
        acc = {"orth": oracle.metric_orth(Qh), "backward": oracle.metric_backward(A_h, Qh, Rh, normA)}
        if name == "grad-c100":
            acc["grad_rel_err"] = grad_error(A_h, ct, dA, m)
        if name == "svd-c50":
            acc["svd_backward"] = oracle.metric_svd_backward(A_h, U.cpu().numpy(), S.cpu().numpy(),
                                                             V.cpu().numpy(), normA)
            acc["orth_U"] = oracle.metric_orth(U.cpu().numpy())
        line["accuracy"] = acc

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(name, A_h, n, args.cpu_sample_rows)

    print(json.dumps(line), flush=True)


def bench_batched(args, dtype):
    """batch512: 512 matrices, m ~ U{2,000..200,000}, n ~ U{4,8,16,32,64}, N(0,1) (FP32: the
    rounding of the same draws); a step is one tsqr_qr_batched call over the whole batch."""
    import torch
    import paper_1301_1071_amd as tsqr
    from paper_1301_1071_amd import _lib
    import workloads

    dev = torch.device("cuda:0")
    f32 = dtype == torch.float32
    es = 4 if f32 else 8
    shapes = workloads.batch_shapes()
    mats = workloads.batch_matrices(shapes, dtype=np.float32 if f32 else np.float64)
    As = [torch.from_numpy(A).to(dev) for A in mats]
    plan = tsqr.BatchPlan(shapes, dtype)
    Qs = [torch.empty_like(A) for A in As]
    Rs = [torch.empty((n, n), dtype=dtype, device=dev) for _, n in shapes]
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    info = torch.zeros(len(As), dtype=torch.int32, device=dev)
    P = tsqr.BatchPlan.pointers
    pa, pq, pr = P(As, dev), P(Qs, dev), P(Rs, dev)

    def step():
        plan.run(pa, pq, pr, ws, info)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.profile_collect()
    _lib.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.profile_enable(False)
    prof = _lib.profile_collect()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # the same call captured once in a graph and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - tg0) * 1e3 / args.steps

    sum_mn = float(sum(m * n for m, n in shapes))
    alg_bytes = 2.0 * es * sum_mn                    # read every A_i, write every Q_i
    value = alg_bytes / (ms_step * 1e-3) / 1e9
    kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
               for k, v in prof.items() if v[1] > 0}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    dom_ms_launch = prof[dom][0] / prof[dom][1]
    launches = prof[dom][1] / args.steps
    if dom == "factor_level0":
        flops = sum(level0_flops(m, n, tsqr.tune_get(dtype, n)[1], form_q=True) for m, n in shapes)
        byts = 2.0 * es * sum_mn
    elif dom == "apply_level0":
        flops, byts = sum(2.0 * m * n * n for m, n in shapes), 2.0 * es * sum_mn
    else:
        flops, byts = 0.0, 2.0 * es * sum_mn
    flops /= launches                                # per launch (one launch per width)
    byts /= launches
    peak_t = FP32_PEAK_TFLOPS if f32 else FP64_PEAK_TFLOPS
    sec = dom_ms_launch * 1e-3
    if flops / byts > peak_t * 1e12 / (HBM_PEAK_GBS * 1e9):
        a = flops / sec / 1e12
        roof = {"bound": "alu", "achieved": a, "peak": peak_t, "unit": "TFLOP/s",
                "frac": a / peak_t, "traffic": None}
    else:
        a = byts / sec / 1e9
        roof = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": a / HBM_PEAK_GBS, "traffic": None}
    roof.update({"kernel": dom, "ms_per_launch": dom_ms_launch})
    per_n = {}
    for (m, n) in shapes:
        per_n.setdefault(n, [0, 0])
        per_n[n][0] += 1
        per_n[n][1] += m
    line = {
        "metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": "batch512" + ("-f32" if f32 else ""), "matrices": len(shapes),
                   "sum_rows": int(sum(m for m, _ in shapes)),
                   "per_width": {str(k): {"count": v[0], "rows": v[1]} for k, v in sorted(per_n.items())},
                   "seed": workloads.SEEDS["batch512"], "algorithmic_bytes": alg_bytes,
                   "launches_per_call": plan.launches},
        "hbm_frac": value / HBM_PEAK_GBS,
        "rows_per_s": sum(m for m, _ in shapes) / (ms_step * 1e-3),
        "graph_ms_per_step": graph_ms,
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_accuracy:
        import oracle
        worst = {"orth": 0.0, "backward": 0.0}
        for k in range(0, len(mats), 64):           # every 64th matrix, full metrics
            A = mats[k].astype(np.float64)
            Q = Qs[k].cpu().numpy().astype(np.float64)
            R = Rs[k].cpu().numpy().astype(np.float64)
            worst["orth"] = max(worst["orth"], oracle.metric_orth(Q))
            worst["backward"] = max(worst["backward"], oracle.metric_backward(A, Q, R))
        line["accuracy"] = worst
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        done, byts = 0, 0.0
        while time.perf_counter() - t0 < 10.0 and done < len(mats):
            A = mats[done].astype(np.float64)
            oracle.tsqr(A, block_rows=1000)
            byts += 2.0 * es * A.shape[0] * A.shape[1]
            done += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": byts / dt / 1e9, "unit": "GB/s",
                                "cores": oracle.max_threads(0), "kind": "oracle",
                                "sample": "first %d of %d matrices, oracle blocks of 1,000 rows, "
                                          "%.1f s" % (done, len(mats), dt)}
    print(json.dumps(line), flush=True)


# HBM bytes per launch of a kernel class, measured with rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (scaled by the copy calibration) for the kernels as they are now; the summaries with the
# commands are in profiles/.  Keyed by (workload, kernel class).
MEASURED_TRAFFIC = {
    ("svd-c50", "factor_level0"): 3.531e9,      # profiles/factor_blk_svd-c50.md
    ("svd-c50", "apply_level0"): 5.161e9,       # profiles/apply_mfma_svd-c50.md
}


def roofline(dom, ms_launch, m, n, plan_op, precision, _lib):
    """Roofline entry for one launch of the dominant kernel class: algorithmic flops and bytes of
    that launch, placed against FP64 peak or HBM bandwidth by their ratio."""
    if dom == "factor_level0":
        b = _lib.plan_levels(plan_op, m, n, precision)[0][1]
        flops, byts = level0_flops(m, n, b, form_q=True), 16.0 * m * n     # read A, write Q1
    elif dom == "apply_level0":
        k = 2 * n if plan_op == "svd" else n
        flops, byts = 2.0 * m * n * k, 8.0 * m * n + 8.0 * m * k          # read Q1, write Q (U)
    elif dom == "bwd_gemm":
        flops, byts = 4.0 * m * n * n, 24.0 * m * n                        # read Q, dQ; write dA
    elif dom == "bwd_gram":
        flops, byts = 2.0 * m * n * n, 16.0 * m * n                        # read dQ, Q
    else:
        flops, byts = 0.0, 16.0 * m * n
    sec = ms_launch * 1e-3
    if flops / byts > FP64_RIDGE:
        a = flops / sec / 1e12
        return {"bound": "alu", "achieved": a, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": a / FP64_PEAK_TFLOPS, "traffic": None}
    a = byts / sec / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": a / HBM_PEAK_GBS, "traffic": None}


def grad_error(A_h, ct, dA, m):
    """Relative error of dA against the oracle's adjoint on the leading rows: the rows of dA depend
    on all of A through the Gram dQ^T Q, so the oracle runs on the full input (bounded cost)."""
    import oracle
    Qo, Ro = oracle.tsqr(A_h, block_rows=8192)
    ref = oracle.qr_backward(Qo, Ro, ct["dQ"], ct["dR"])
    got = dA.cpu().numpy()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def cpu_baseline(name, A_h, n, sample_rows, min_seconds=10.0):
    """The oracle as it stands, on the leading rows of the same workload, repeated until about
    ten seconds of CPU work have been timed; reports the mean rate."""
    import oracle
    import workloads
    cfg = workloads.CONFIGS[name]
    threads = oracle.max_threads(0)
    default_rows = {"grad-c100": 250_000}.get(name, A_h.shape[0])
    ms = min(A_h.shape[0], sample_rows or default_rows)
    As = np.ascontiguousarray(A_h[:ms])
    ct = workloads.cotangents(ms, n) if name == "grad-c100" else None
    per_pass = {"svd-c50": 3, "grad-c100": 5}.get(name, 2) * 8.0 * ms * n
    reps, dt = 0, 0.0
    while dt < min_seconds:
        t0 = time.perf_counter()
        if name == "svd-c50":
            oracle.tsqr_svd(As, block_rows=cfg["block_rows"], want_qr=True)
        elif name == "grad-c100":
            Qo, Ro = oracle.tsqr(As, block_rows=cfg["block_rows"])
            oracle.qr_backward(Qo, Ro, ct["dQ"], ct["dR"])
        else:
            oracle.tsqr(As, block_rows=cfg["block_rows"])
        dt += time.perf_counter() - t0
        reps += 1
    return {"value": per_pass * reps / dt / 1e9, "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d of %d rows, oracle blocks of %d rows, %d passes in %.1f s" % (
                ms, A_h.shape[0], cfg["block_rows"], reps, dt)}


if __name__ == "__main__":
    main()
