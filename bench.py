"""Benchmark: semi-discrete OT solve (MAK reconstruction hot path) on one GPU.

One step = one complete damped-Newton solve from psi = 0 to
max_i |V_i - m_i| / m_i <= tol on a synthetic input resident in HBM: grid
build, every Laguerre cell pass (Newton and line-search trials), Hessian
assembly, Jacobi-PCG, and the outputs (psi, centroids, displacements).

value = Laguerre cells computed per second over the timed solves
        (cells = N x cell passes); ms_per_step = solve time.

Also reported: the other precision path on the same input, the roofline of
the dominant kernel (HIP-event durations of its launches in the timed region,
counted work from a separate counting solve), and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Laguerre cells/s + OT solve time at 128^3, FP64 vs mixed; served p50/p99"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6

WORKLOADS = {
    # name: (generator kwargs, tol, default precision)
    "clustered_128": (dict(kind="clustered", n=128, rms=3.0, smooth=1.0, frac=0.2, n_clumps=2000,
                           a=0.5, seed=3), 1e-6, "fp64"),
    "zeldovich_64": (dict(kind="zeldovich", n=64, rms=1.0, smooth=1.0, seed=2), 1e-6, "fp64"),
    "zeldovich_16": (dict(kind="zeldovich", n=16, rms=0.3, smooth=2.0, seed=1), 1e-6, "fp64"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_input(spec):
    import workloads
    s = dict(spec)
    kind = s.pop("kind")
    if kind == "clustered":
        return workloads.clustered(**s)
    return workloads.zeldovich(**s)


def timed_solves(mak, x_dev, L, tol, precision, steps, warmup, cg_rtol, verbose=0):
    import torch
    ctx = mak.Context(0, precision, cg_rtol=cg_rtol, verbose=verbose)
    for w in range(warmup):
        _, _, _, info = ctx.solve(x_dev, L, tol)
        log(f"[bench] warmup {w} {precision}: {info}")
    ctx.profile_enable(timing=True, counting=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(steps):
        _, _, _, info = ctx.solve(x_dev, L, tol)
        infos.append(info)
        log(f"[bench] step {k} {precision}: newton={info['newton_iters']} passes={info['cell_passes']} "
            f"cg={info['cg_iters_total']} err={info['final_err']:.2e} t={info['seconds']:.3f}s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    # counting solve (outside the timed region): work per clip launch
    ctx.profile_enable(timing=True, counting=True)
    ctx.solve(x_dev, L, tol)
    cprof = ctx.profile_read()
    ctx.close()
    return t1 - t0, infos, prof, cprof


def roofline(prof, cprof):
    kern = {k: v for k, v in prof.items() if not k.startswith("_") and k not in ("pcg_solve",)}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    v = kern[dom]
    avg_ms = v["total_ms"] / max(v["launches"], 1)
    c = cprof.get(dom, v)
    per_launch_flops = c["flops"] / max(c["launches"], 1)
    per_launch_bytes = c["bytes"] / max(c["launches"], 1)
    if dom.startswith("clip"):
        achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
        out = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
               "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": None,
               "avg_launch_ms": avg_ms, "launches": v["launches"],
               "flops_per_launch": per_launch_flops, "bytes_per_launch": per_launch_bytes,
               "hbm_GBs_algorithmic": per_launch_bytes / (avg_ms * 1e-3) / 1e9}
    else:
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        out = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
               "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
               "avg_launch_ms": avg_ms, "launches": v["launches"],
               "bytes_per_launch": per_launch_bytes}
    share = {k: round(kern[k]["total_ms"], 3) for k in kern}
    return out, share


def cpu_baseline(x, L, seconds):
    """The oracle as it stands, on a bounded sample of cells of the same
    workload at psi = 0 (its per-cell cost is O(27 N))."""
    import numpy as np

    import oracle
    threads = min(os.cpu_count() or 1, 16)
    N = x.shape[0]
    psi = np.zeros(N)
    rng = np.random.default_rng(0)
    probe = max(threads, 8)
    idx = rng.choice(N, probe, replace=False)
    t0 = time.perf_counter()
    oracle.cells(x, psi, L, idx=idx, threads=threads)
    dt = time.perf_counter() - t0
    per_cell = dt / probe
    m = int(max(probe, min(N, seconds / max(per_cell, 1e-9))))
    idx = rng.choice(N, m, replace=False)
    t0 = time.perf_counter()
    oracle.cells(x, psi, L, idx=idx, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} random cells of the same {N}-site input at psi=0 "
                      f"(one cell pass, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="clustered_128", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--compare", default="mixed", choices=["fp64", "mixed", "none"],
                    help="also time the other precision path (default: the other one if built)")
    ap.add_argument("--cg-rtol", type=float, default=1e-3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "domain decomposition is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2110_08868_amd as mak

    spec, tol, default_prec = WORKLOADS[args.workload]
    precision = args.precision or default_prec
    L = 1.0
    log(f"[bench] generating {args.workload} ...")
    x = make_input(spec)
    N = x.shape[0]
    x_dev = torch.from_numpy(x).cuda()
    torch.cuda.synchronize()

    secs, infos, prof, cprof = timed_solves(mak, x_dev, L, tol, precision, args.steps, args.warmup,
                                            args.cg_rtol, int(args.verbose))
    passes = sum(i["cell_passes"] for i in infos)
    value = N * passes / secs
    rl, share = roofline(prof, cprof)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "L": L, "tol": tol, "precision": precision,
                   **{k: v for k, v in spec.items()}, "cg_rtol": args.cg_rtol},
        "solve": {"seconds_median": float(np.median([i["seconds"] for i in infos])),
                  "newton_iters": infos[-1]["newton_iters"], "cell_passes": infos[-1]["cell_passes"],
                  "cg_iters": infos[-1]["cg_iters_total"], "final_err": infos[-1]["final_err"]},
        "kernel_ms_total": share,
        "work_counters_per_solve": cprof.get("_counters"),
        "roofline": rl,
    }
    other = args.compare
    if other is None:
        other = "none"
    if other not in ("none", precision):
        s2, inf2, p2, c2 = timed_solves(mak, x_dev, L, tol, other, max(1, args.steps), 0, args.cg_rtol)
        res[other] = {"cells_per_s": N * sum(i["cell_passes"] for i in inf2) / s2,
                      "ms_per_solve": s2 / len(inf2) * 1e3,
                      "newton_iters": inf2[-1]["newton_iters"], "final_err": inf2[-1]["final_err"]}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(x, L, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
