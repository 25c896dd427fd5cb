#!/usr/bin/env python3
"""Benchmark of direct TSQR on one MI355X.

A step is one pass of the whole hot path over one synthetic input already resident in HBM.  The
headline workload (svd-c50: A = G diag(s) V^T, 4,000,000 x 50, s = logspace(0,-12,50)) is one
tsqr_svd call returning Q, R, U, S and V; `value` is the whole-job rate in algorithmic GB/s
(A read once, Q and U written once: 8 m n bytes each).

Prints ONE JSON line:
  value / ms_per_step   wall clock over the timed steps; the library's event profiler records
                        only the dominant kernel class inside that region (two events per
                        launch of that class), found by an untimed profiled pass before it;
  kernels               per-class ms per step and launches (the untimed profiled pass);
  roofline              the dominant class: algorithmic flops or bytes of one launch (the
                        paper-method counts: Householder 2 b n^2 - 2/3 n^3 per b-row panel,
                        2 rows n k per step-3 product) over its mean launch time from the
                        events of the timed region; `traffic` from profiles/traffic.json when
                        the kernel's sources still hash to the profiled ones, else null;
  accuracy              Sec. I-B metrics from the library's compensated GPU Gram kernels;
  cpu_baseline          the CPU oracle on a bounded sample, on this host's cores;
  forms                 the other workloads on the same GPU: qr-small (graph replays),
                        mixed-c25 (FP64 vs FP32 vs FP32 + refinement), batch512 (FP64 / FP32,
                        per width), grad-c100 (forward vs adjoint), stability (Sec. IV:
                        ||Q^T Q - I|| of direct TSQR and the comparison methods per condition),
                        paper_scale (600M x 25 QR and 150M x 100 R, Sec. V shapes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64, matrix and vector alike
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 matrix
METRIC = "TSQR GB/s and % HBM roofline vs plain FP64; ||Q^T Q-I||, backward rel err"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="svd-c50",
                    choices=["svd-c50", "qr-small", "mixed-c25", "grad-c100"])
    ap.add_argument("--rows", type=int, default=0, help="override m (same recipe and seed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="only the headline workload")
    ap.add_argument("--cpu-sample-rows", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


# ----------------------------------------------------------------------------- algorithmic counts
def hh_flops(b, n):
    """Householder QR of one b x n block (Sec. III-A): 2 b n^2 - 2/3 n^3 (b >= n)."""
    if b >= n:
        return 2.0 * b * n * n - 2.0 / 3.0 * n ** 3
    return 2.0 * b * b * n - 2.0 / 3.0 * b ** 3


def level_flops(rows, n, b):
    full, tail = divmod(rows, b)
    return full * hh_flops(b, n) + (hh_flops(tail, n) if tail else 0.0)


def class_model(cls, plan, m, n, k, precision, launches):
    """(flops, bytes, fp32) of ONE launch of kernel class `cls` by the paper-method counts."""
    fp32 = precision != "fp64"
    lv = plan
    if cls == "factor_level0":
        return level_flops(m, n, lv[0][1]), 8.0 * m * n, fp32
    if cls == "factor_tree" and len(lv) > 1:
        f = sum(level_flops(r, n, b) for r, b in lv[1:])
        by = sum(8.0 * r * n for r, _ in lv[1:])
        return f / launches, by / launches, False
    if cls == "apply_level0":
        es = 4.0 if fp32 else 8.0
        return 2.0 * m * n * k, es * m * n + 8.0 * m * k, fp32
    if cls == "apply_tree" and len(lv) > 1:
        f = sum(2.0 * r * n * k for r, _ in lv[1:])
        by = sum(16.0 * r * n for r, _ in lv[1:])
        return f / launches, by / launches, False
    if cls == "refine":
        # two or three passes reading A, one writing Q (the second Gram pass may be skipped)
        return 4.0 * m * n * n / launches, 24.0 * m * n / launches, False
    if cls == "bwd_gram":
        return 2.0 * m * n * n / launches, 16.0 * m * n / launches, False
    if cls == "bwd_gemm":
        return 4.0 * m * n * n / launches, 32.0 * m * n / launches, False
    return None


def roofline(cls, ms_launch, model):
    if model is None:
        return {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None}
    flops, byts, fp32 = model
    peak_t = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
    ridge = peak_t * 1e12 / (HBM_PEAK_GBS * 1e9)
    sec = ms_launch * 1e-3
    if flops / byts > ridge:
        a = flops / sec / 1e12
        return {"bound": "mfma", "achieved": a, "peak": peak_t, "unit": "TFLOP/s",
                "frac": a / peak_t, "traffic": None, "flops_per_launch": flops}
    a = byts / sec / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": a / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": byts}


def src_sha16(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, cls):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if the
    kernel's sources are unchanged since it was taken; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            tab = json.load(fh)
    except (OSError, ValueError):
        return None
    e = tab.get("%s:%s" % (workload, cls))
    if not e:
        return None
    if src_sha16(e["sources"]) != e["src_sha16"]:
        return None
    return e["bytes_per_launch"]


# ----------------------------------------------------------------------------- timing helpers
def run_timed(step, steps, warmup, lib_mod, classes_all):
    """Untimed profiled pass (all classes) -> breakdown and dominant class; then the timed region
    with events around the dominant class only.  Returns (ms_per_step, kernels, dom, ms_launch)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lib_mod.profile_collect()
    lib_mod.profile_set_mask(None)
    lib_mod.profile_enable(True)
    prof_steps = max(1, min(steps, 5))
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    lib_mod.profile_enable(False)
    prof = lib_mod.profile_collect()
    kernels = {k: {"ms_per_step": v[0] / prof_steps, "launches_per_step": v[1] / prof_steps}
               for k, v in prof.items() if v[1] > 0}
    dom = max(kernels, key=lambda c: kernels[c]["ms_per_step"])
    lib_mod.profile_set_mask([dom])
    lib_mod.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib_mod.profile_enable(False)
    lib_mod.profile_set_mask(None)
    p2 = lib_mod.profile_collect()
    ms_launch = p2[dom][0] / max(1, p2[dom][1])
    return (t1 - t0) * 1e3 / steps, kernels, dom, ms_launch, p2[dom][1] / steps


def wall_ms(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def graph_replay_ms(step, replays=200):
    """Capture `step` in a HIP graph; median of `replays` event-timed replays."""
    import torch
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                                     # warm the allocator outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    ts = []
    for _ in range(replays):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), g


# ----------------------------------------------------------------------------- headline workload
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
    cfg = workloads.CONFIGS[name]
    m = args.rows or cfg["m"]
    n = cfg["n"]
    A_h = workloads.config_matrix(name, m=m)
    A = torch.from_numpy(A_h).to(dev)
    torch.cuda.synchronize()
    info = torch.zeros(1, dtype=torch.int32, device=dev)

    if name == "svd-c50":
        U = torch.empty((m, n), dtype=torch.float64, device=dev)
        S = torch.empty((n,), dtype=torch.float64, device=dev)
        V = torch.empty((n, n), dtype=torch.float64, device=dev)
        Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(tsqr.workspace_bytes("svd", m, n), dtype=torch.uint8, device=dev)

        def step():
            tsqr.svd(A, want_qr=True, ws=ws, out=(U, S, V, Q, R), check_info=False, info=info)
        alg_bytes = 3 * 8.0 * m * n          # read A, write Q and U
        desc = "direct TSQR + SVD (Q, R, U, S, V), A = G diag(logspace(0,-12)) V^T"
        precision, plan_op, k = "fp64", "svd", 2 * n
    elif name == "grad-c100":
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
            tsqr.qr(A, ws=ws, out=(Q, R), check_info=False, info=info)
            tsqr.qr_backward(A, dQ, dR, ws=ws, out=dA, check_info=False)
        alg_bytes = 2 * 8.0 * m * n + 3 * 8.0 * m * n   # fwd: A, Q; bwd: A, dQ, dA
        desc = "direct TSQR forward (Q, R) + closed-form QR adjoint (dA), Q recomputed from A"
        precision, plan_op, k = "fp64", "qr", n
    else:
        precision = "fp64" if name == "qr-small" else "fp32_refined"
        Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(tsqr.workspace_bytes("qr", m, n, precision), dtype=torch.uint8, device=dev)

        def step():
            tsqr.qr(A, precision=precision, ws=ws, out=(Q, R), check_info=False, info=info)
        alg_bytes = 2 * 8.0 * m * n          # read A, write Q
        desc = "direct TSQR (Q, R)" + (" FP32 panels + FP64 refinement" if precision != "fp64" else "")
        plan_op, k = "qr", n

    if args.copy_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms_step, kernels, dom, dom_ms, dom_launches = run_timed(step, args.steps, args.warmup, _lib, None)
    value = alg_bytes / (ms_step * 1e-3) / 1e9
    plan = _lib.plan_levels(plan_op, m, n, "fp32" if precision != "fp64" else "fp64")
    roof = roofline(dom, dom_ms, class_model(dom, plan, m, n, k, precision, dom_launches))
    roof["kernel"] = dom
    roof["ms_per_launch"] = dom_ms
    if args.rows == 0:
        roof["traffic"] = measured_traffic(name, dom)

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
        "flops_2mn2_per_s": 2.0 * m * n * n / (ms_step * 1e-3),
        "roofline": roof,
        "kernels": kernels,
        "tree_levels": [{"rows": r, "panel_rows": b} for r, b in plan],
    }

    if not args.no_accuracy:
        acc = {"info": int(info.item())}
        normA = tsqr.metric_norm2(A)
        acc["orth"] = tsqr.metric_orth(Q)
        acc["backward"] = tsqr.metric_residual(A, Q, R) / normA
        if name == "svd-c50":
            B = S[:, None] * V.t()
            acc["svd_backward"] = tsqr.metric_residual(A, U, B.contiguous()) / normA
            acc["orth_U"] = tsqr.metric_orth(U)
            acc["orth_V"] = float(np.linalg.norm(V.cpu().numpy().T @ V.cpu().numpy() - np.eye(n), 2))
        if name == "grad-c100":
            acc["dA_finite"] = bool(torch.isfinite(dA).all())
        line["accuracy"] = acc

    if not args.no_forms and name == "svd-c50" and args.rows == 0:
        del A, U, Q, ws
        torch.cuda.empty_cache()
        line["forms"] = bench_forms(args, dev)

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(name, A_h, n, args.cpu_sample_rows)

    print(json.dumps(line), flush=True)


# ----------------------------------------------------------------------------- the other forms
def bench_forms(args, dev):
    out = {}
    for fn in (form_qr_small, form_mixed, form_batched, form_grad, form_stability,
               form_paper_scale):
        t0 = time.perf_counter()
        try:
            out[fn.__name__[5:]] = fn(args, dev)
        except Exception as e:        # a failing form is reported, not hidden
            out[fn.__name__[5:]] = {"error": "%s: %s" % (type(e).__name__, e)}
        out[fn.__name__[5:]]["bench_s"] = time.perf_counter() - t0
        import torch
        torch.cuda.empty_cache()
    return out


def form_qr_small(args, dev):
    """qr-small (100,000 x 10): eager ms, and the median of 200 graph replays (launch-bound)."""
    import torch
    import paper_1301_1071_amd as tsqr
    import workloads
    m, n = workloads.CONFIGS["qr-small"]["m"], workloads.CONFIGS["qr-small"]["n"]
    A = torch.from_numpy(workloads.config_matrix("qr-small")).to(dev)
    Q = torch.empty((m, n), dtype=torch.float64, device=dev)
    R = torch.empty((n, n), dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(tsqr.workspace_bytes("qr", m, n), dtype=torch.uint8, device=dev)

    def step():
        tsqr.qr(A, ws=ws, out=(Q, R), check_info=False, info=info)
    eager = wall_ms(step, 50, 5)
    Q0 = Q.clone()
    gms, g = graph_replay_ms(step)
    torch.cuda.synchronize()
    by = 16.0 * m * n
    return {"m": m, "n": n, "eager_ms": eager, "graph_ms_median200": gms,
            "graph_GBps": by / (gms * 1e-3) / 1e9, "graph_rows_per_s": m / (gms * 1e-3),
            "graph_matches_eager": bool(torch.equal(Q, Q0)),
            "orth": tsqr.metric_orth(Q),
            "backward": tsqr.metric_residual(A, Q, R) / tsqr.metric_norm2(A)}


def form_mixed(args, dev):
    """mixed-c25 (16,000,000 x 25, cond 1e4): the plain FP64 form, the FP32 form (before
    refinement) and FP32 + the FP64 refinement, on the same input."""
    import torch
    import paper_1301_1071_amd as tsqr
    from paper_1301_1071_amd import _lib
    import workloads
    c = workloads.CONFIGS["mixed-c25"]
    m, n = c["m"], c["n"]
    A = torch.from_numpy(workloads.config_matrix("mixed-c25")).to(dev)
    Q = torch.empty((m, n), dtype=torch.float64, device=dev)
    R = torch.empty((n, n), dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    normA = tsqr.metric_norm2(A)
    res = {"m": m, "n": n}
    for prec in ("fp64", "fp32", "fp32_refined"):
        ws = torch.empty(tsqr.workspace_bytes("qr", m, n, prec), dtype=torch.uint8, device=dev)

        def step():
            tsqr.qr(A, precision=prec, ws=ws, out=(Q, R), check_info=False, info=info)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        _lib.profile_collect()
        _lib.profile_enable(True)
        ms = wall_ms(step, 5, 0)
        _lib.profile_enable(False)
        prof = _lib.profile_collect()
        res[prec] = {"ms": ms, "GBps": 16.0 * m * n / (ms * 1e-3) / 1e9,
                     "kernels_ms": {k: v[0] / 5 for k, v in prof.items() if v[1]},
                     "info": int(info.item()),
                     "orth": tsqr.metric_orth(Q),
                     "backward": tsqr.metric_residual(A, Q, R) / normA}
        del ws
        torch.cuda.empty_cache()
    return res


def form_batched(args, dev):
    """batch512: 512 ragged matrices in one launch sequence, FP64 and FP32; eager and graph ms,
    and per width class (each class run as its own plan)."""
    import torch
    import paper_1301_1071_amd as tsqr
    import workloads
    shapes = workloads.batch_shapes()
    res = {"matrices": len(shapes), "sum_rows": int(sum(m for m, _ in shapes))}
    for dt, npdt, es, key in ((torch.float64, np.float64, 8, "fp64"),
                              (torch.float32, np.float32, 4, "fp32")):
        mats = workloads.batch_matrices(shapes, dtype=npdt)
        As = [torch.from_numpy(a).to(dev) for a in mats]
        del mats

        def run_plan(idx):
            sub = [shapes[i] for i in idx]
            plan = tsqr.BatchPlan(sub, dt)
            Qs = [torch.empty_like(As[i]) for i in idx]
            Rs = [torch.empty((shapes[i][1], shapes[i][1]), dtype=dt, device=dev) for i in idx]
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
            info = torch.zeros(len(idx), dtype=torch.int32, device=dev)
            P = tsqr.BatchPlan.pointers
            pa, pq, pr = P([As[i] for i in idx], dev), P(Qs, dev), P(Rs, dev)

            def step():
                plan.run(pa, pq, pr, ws, info)
            ms = wall_ms(step, 5, 2)
            gms, _ = graph_replay_ms(step, replays=10)
            by = 2.0 * es * sum(m * n for m, n in sub)
            r = {"ms": ms, "graph_ms": gms, "GBps": by / (ms * 1e-3) / 1e9,
                 "graph_GBps": by / (gms * 1e-3) / 1e9, "launches": plan.launches,
                 "info_nonzero": int(torch.count_nonzero(info).item())}
            return r, Qs, Rs
        allr, Qs, Rs = run_plan(list(range(len(shapes))))
        worst_o, worst_b = 0.0, 0.0
        for i in range(0, len(shapes), 64):
            Qd = Qs[i].double()
            worst_o = max(worst_o, tsqr.metric_orth(Qd))
            worst_b = max(worst_b, tsqr.metric_residual(As[i].double(), Qd, Rs[i].double())
                          / tsqr.metric_norm2(As[i].double()))
        allr["orth_worst_every64"] = worst_o
        allr["backward_worst_every64"] = worst_b
        del Qs, Rs
        per = {}
        for w in sorted({n for _, n in shapes}):
            idx = [i for i, (_, n) in enumerate(shapes) if n == w]
            r, q, rr = run_plan(idx)
            del q, rr
            per[str(w)] = {"count": len(idx), "rows": int(sum(shapes[i][0] for i in idx)), **r}
        allr["per_width"] = per
        res[key] = allr
        del As
        torch.cuda.empty_cache()
    return res


def form_grad(args, dev):
    """grad-c100 (1,000,000 x 100): forward QR vs its adjoint, forward SVD vs its adjoint."""
    import torch
    import paper_1301_1071_amd as tsqr
    import workloads
    c = workloads.CONFIGS["grad-c100"]
    m, n = c["m"], c["n"]
    A = torch.from_numpy(workloads.config_matrix("grad-c100")).to(dev)
    ct = workloads.cotangents(m, n)
    dQ, dR, dU, dS, dV = (torch.from_numpy(ct[k]).to(dev) for k in ("dQ", "dR", "dU", "dS", "dV"))
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    Q = torch.empty((m, n), dtype=torch.float64, device=dev)
    R = torch.empty((n, n), dtype=torch.float64, device=dev)
    dA = torch.empty((m, n), dtype=torch.float64, device=dev)
    ws = torch.empty(max(tsqr.workspace_bytes(o, m, n) for o in
                         ("qr", "svd", "qr_backward", "svd_backward")), dtype=torch.uint8, device=dev)
    res = {"m": m, "n": n}
    res["qr_forward_ms"] = wall_ms(lambda: tsqr.qr(A, ws=ws, out=(Q, R), check_info=False,
                                                   info=info), 5, 2)
    res["qr_backward_ms"] = wall_ms(lambda: tsqr.qr_backward(A, dQ, dR, ws=ws, out=dA,
                                                             check_info=False), 5, 2)
    U = torch.empty((m, n), dtype=torch.float64, device=dev)
    S = torch.empty((n,), dtype=torch.float64, device=dev)
    V = torch.empty((n, n), dtype=torch.float64, device=dev)
    res["svd_forward_ms"] = wall_ms(lambda: tsqr.svd(A, ws=ws, out=(U, S, V, None, None),
                                                     check_info=False, info=info), 5, 2)
    res["svd_backward_ms"] = wall_ms(lambda: tsqr.svd_backward(A, dU, dS, dV, ws=ws, out=dA,
                                                               check_info=False), 5, 2)
    res["qr_backward_GBps"] = 24.0 * m * n / (res["qr_backward_ms"] * 1e-3) / 1e9
    res["qr_forward_GBps"] = 16.0 * m * n / (res["qr_forward_ms"] * 1e-3) / 1e9
    res["dA_finite"] = bool(torch.isfinite(dA).all())
    return res


def form_stability(args, dev):
    """The stability experiment of Sec. IV on the GPU: ||Q^T Q - I||_2 and the backward error of
    direct TSQR and the comparison methods (Cholesky QR, indirect TSQR with Q = A R^{-1}, each
    with and without one step of iterative refinement) on 100,000 x 10 matrices
    A = G diag(logspace(0, -c, 10)) V^T, c = 0, 2, ..., 16.  A method that breaks down (Cholesky
    of a Gram matrix that is not numerically positive definite) is reported as "breakdown"."""
    import torch
    import paper_1301_1071_amd as tsqr
    import workloads
    m, n = 100_000, 10
    rows = {}
    for c in range(0, 17, 2):
        A = torch.from_numpy(workloads.spectrum_matrix(m, n, float(c), seed=700 + c)[0]).to(dev)
        normA = tsqr.metric_norm2(A)
        r = {}
        Q, R = tsqr.qr(A, check_info=False)
        r["direct"] = {"orth": tsqr.metric_orth(Q), "backward": tsqr.metric_residual(A, Q, R) / normA,
                       "ms": wall_ms(lambda: tsqr.qr(A, out=(Q, R), check_info=False), 5, 1)}
        for meth in ("cholqr", "cholqr_ir", "indirect", "indirect_ir"):
            Q, R, info = tsqr.qr_indirect(A, meth)
            ms = wall_ms(lambda: tsqr.qr_indirect(A, meth, out=(Q, R)), 5, 1)
            Q, R, info = tsqr.qr_indirect(A, meth, out=(Q, R))
            torch.cuda.synchronize()
            if int(info.item()) == -4:
                r[meth] = {"orth": "breakdown", "backward": None, "ms": ms}
            else:
                r[meth] = {"orth": tsqr.metric_orth(Q),
                           "backward": tsqr.metric_residual(A, Q, R) / normA, "ms": ms}
        rows["1e%d" % c] = r
    return {"m": m, "n": n, "by_cond": rows}


def form_paper_scale(args, dev):
    """Two of the paper's own shapes (Sec. V) on the one GPU, inputs built on the device:
    600,000,000 x 25 QR (level-0 factors kept in Q, so that A, Q and the workspace fit in HBM)
    and SVD (U in place of Q), 150,000,000 x 100 R, and its full QR by the row-chunked driver, each the mean of 3 timed
    calls after one warm-up, with the compensated Sec. I-B metrics.  The paper's Hadoop job times for the same shapes (Tables VI
    and I, a 40-core cluster reading HDFS) are quoted as context."""
    import torch
    import paper_1301_1071_amd as tsqr
    import workloads
    res = {}
    c = workloads.PAPER_SCALE["paper-600m"]
    m, n = c["m"], c["n"]
    wsb = tsqr.workspace_bytes("qr", m, n, reuse_output=True)
    free, _ = torch.cuda.mem_get_info()
    if free < 16 * m * n + wsb + (2 << 30):
        res["qr_600m_x_25"] = {"skipped": "%.0f GiB free" % (free / 2 ** 30)}
    else:
        A = torch.empty((m, n), dtype=torch.float64, device=dev)
        workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-600m"])
        Q = torch.empty_like(A)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        ms = wall_ms(lambda: tsqr.qr(A, ws=ws, out=(Q, R), check_info=False, info=info,
                                     reuse_output=True), 3, 1)
        del ws
        res["qr_600m_x_25"] = {
            "m": m, "n": n, "ms": ms, "GBps": 16.0 * m * n / (ms * 1e-3) / 1e9,
            "flops_2mn2_per_s": 2.0 * m * n * n / (ms * 1e-3), "info": int(info.item()),
            "orth": tsqr.metric_orth(Q),
            "backward": tsqr.metric_residual(A, Q, R) / float(torch.linalg.matrix_norm(R.cpu(), 2)),
            "paper_job_s": {"python_table6": 1910, "cxx_table1": 1482}}
        del A, Q
        torch.cuda.empty_cache()
    # the SVD variant of the same shape: U out of step 3 in place of Q (level-0 factors in U)
    wsb = tsqr.workspace_bytes("svd", m, n, reuse_output=True)
    free, _ = torch.cuda.mem_get_info()
    if free < 16 * m * n + wsb + (2 << 30):
        res["svd_600m_x_25"] = {"skipped": "%.0f GiB free" % (free / 2 ** 30)}
    else:
        A = torch.empty((m, n), dtype=torch.float64, device=dev)
        workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-600m"])
        U = torch.empty_like(A)
        S = torch.empty((n,), dtype=torch.float64, device=dev)
        V = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        ms = wall_ms(lambda: tsqr.svd(A, ws=ws, out=(U, S, V, None, None), check_info=False,
                                      info=info, reuse_output=True), 3, 1)
        del ws
        res["svd_600m_x_25"] = {
            "m": m, "n": n, "ms": ms, "GBps": 16.0 * m * n / (ms * 1e-3) / 1e9,
            "info": int(info.item()), "orth_U": tsqr.metric_orth(U),
            "svd_backward": tsqr.metric_residual(A, U, (S[:, None] * V.t()).contiguous())
                            / float(S[0])}
        del A, U
        torch.cuda.empty_cache()
    c = workloads.PAPER_SCALE["paper-150m"]
    m, n = c["m"], c["n"]
    wsb = tsqr.workspace_bytes("r", m, n)
    free, _ = torch.cuda.mem_get_info()
    if free < 8 * m * n + wsb + (4 << 30):
        res["r_150m_x_100"] = {"skipped": "%.0f GiB free" % (free / 2 ** 30)}
    else:
        A = torch.empty((m, n), dtype=torch.float64, device=dev)
        workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-150m"])
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        ms = wall_ms(lambda: tsqr.r(A, ws=ws, check_info=False), 3, 1)
        R = tsqr.r(A, ws=ws).cpu().numpy()
        del ws
        G = tsqr.metric_gram(2, A).cpu().numpy()
        res["r_150m_x_100"] = {
            "m": m, "n": n, "ms": ms, "GBps": 8.0 * m * n / (ms * 1e-3) / 1e9,
            "gram_err": float(np.max(np.abs(np.linalg.eigvalsh(R.T @ R - G)))
                              / np.max(np.linalg.eigvalsh(G))),
            "paper_job_s_qr": {"python_table6": 2154, "cxx_table1": 1503}}
        del A
        torch.cuda.empty_cache()
    # the full QR of the same shape, in 15,000,000-row chunks (one more tree level)
    h = 15_000_000
    wsb = tsqr.qr_chunked_workspace_bytes(m, n, h)
    free, _ = torch.cuda.mem_get_info()
    if free < 16 * m * n + wsb + (2 << 30):
        res["qr_150m_x_100_chunked"] = {"skipped": "%.0f GiB free" % (free / 2 ** 30)}
    else:
        A = torch.empty((m, n), dtype=torch.float64, device=dev)
        workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-150m"])
        Q = torch.empty_like(A)
        R = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        ms = wall_ms(lambda: tsqr.qr_chunked(A, h, ws=ws, out=(Q, R), check_info=False,
                                             info=info), 3, 1)
        del ws
        res["qr_150m_x_100_chunked"] = {
            "m": m, "n": n, "chunk_rows": h, "ms": ms, "GBps": 16.0 * m * n / (ms * 1e-3) / 1e9,
            "info": int(info.item()), "orth": tsqr.metric_orth(Q),
            "backward": tsqr.metric_residual(A, Q, R) / float(torch.linalg.matrix_norm(R.cpu(), 2)),
            "paper_job_s": {"python_table6": 2154, "cxx_table1": 1503}}
        del A, Q
        torch.cuda.empty_cache()
    return res


# ----------------------------------------------------------------------------- CPU baseline
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
