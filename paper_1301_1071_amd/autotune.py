"""Autotuner of the batched form's panel heights (run on the GPU).

For every width class (n = 4, 8, 16, 32, 64) and element type it times each usable register-panel
variant (`tune_variants`) on a seeded batch of matrices of that width with m ~ U{2,000..200,000}
(the batched workload's row distribution), takes the median of several timed calls of the whole
batched factorization, and records the fastest variant in ``tune_table.json``:

    python -m paper_1301_1071_amd.autotune [--out PATH] [--count 64] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

from . import tsqr
from .tuning import TABLE

WIDTHS = (4, 8, 16, 32, 64)


def time_variant(As, dtype, variant, n, reps):
    tsqr.tune_set(dtype, n, variant)
    plan = tsqr.BatchPlan([tuple(A.shape) for A in As], dtype)
    dev = As[0].device
    Qs = [torch.empty_like(A) for A in As]
    Rs = [torch.empty((n, n), dtype=dtype, device=dev) for _ in As]
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    info = torch.zeros(len(As), dtype=torch.int32, device=dev)
    pa, pq, pr = (tsqr.BatchPlan.pointers(x, dev) for x in (As, Qs, Rs))
    plan.run(pa, pq, pr, ws, info)          # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run(pa, pq, pr, ws, info)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    if int(torch.count_nonzero(info)) != 0:
        raise RuntimeError("autotune: nonzero info for n=%d variant %d" % (n, variant))
    return float(np.median(times))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1301107199)
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    g = np.random.default_rng(args.seed)
    entries = []
    for dtype, tag in ((torch.float64, "f64"), (torch.float32, "f32")):
        for n in WIDTHS:
            ms = g.integers(2000, 200_001, size=args.count)
            As = [torch.from_numpy(g.standard_normal((int(m), n))).to(dev, dtype) for m in ms]
            heights = tsqr.tune_variants(dtype, n)
            res = {}
            for v, b in enumerate(heights):
                if b:
                    res[v] = time_variant(As, dtype, v, n, args.reps)
            best = min(res, key=res.get)
            tsqr.tune_set(dtype, n, best)
            entries.append({"dtype": tag, "n": n, "variant": best, "panel_rows": heights[best],
                            "ms": {str(heights[v]) + "/v" + str(v): t for v, t in res.items()},
                            "batch": args.count})
            print("autotune %s n=%d: %s -> variant %d (%d rows)" % (
                tag, n, {heights[v]: round(t, 3) for v, t in res.items()}, best, heights[best]),
                flush=True)
            del As
    table = {"version": 1, "device": torch.cuda.get_device_name(dev), "entries": entries}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
