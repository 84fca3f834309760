"""Benchmark: semi-discrete OT solve (MAK reconstruction hot path) on one GPU.

One step = one complete damped-Newton solve from psi = 0 to
max_i |V_i - m_i| / m_i <= tol on a synthetic input resident in HBM: grid
build, every Laguerre cell pass (Newton and line-search trials), Hessian
assembly, Jacobi-PCG, and the outputs (psi, centroids, displacements).

value = Laguerre cells computed per second over the timed solves
        (cells = N x cell passes); ms_per_step = solve time.

Also reported: the other precision path on the same input, the roofline of
the dominant kernel (HIP-event durations of its launches in the timed region,
counted work from a separate counting solve), the Legendre transform of the
solved weights on a mesh of N nodes (the initial potential and the location
of every node), the Zel'dovich deposit of the solved cells and the power
spectrum of that density, serving, and the CPU oracle timed on a bounded
sample of the same workload.
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
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2110_08868_amd", "csrc")


# the sources each timed kernel is built from (its file and the headers it
# includes)
KERNEL_SOURCES = {
    "clip": ["clip.hip", "engine.h", "common.h", "gridkey.h", "profile.h"],
    "spmv": ["pcg.hip", "engine.h", "common.h", "profile.h"],
    "locate": ["locate.hip", "engine.h", "common.h", "gridkey.h", "profile.h"],
    "deposit": ["locate.hip", "engine.h", "common.h", "gridkey.h", "profile.h"],
    "shell_bin": ["power.hip", "engine.h", "common.h", "profile.h"],
}


def kernel_source_hash(kernel: str = "clip") -> str:
    """sha256 over the HIP sources of a kernel: measured HBM traffic is only
    reported for the kernel code it was taken on."""
    import hashlib
    files = KERNEL_SOURCES["clip" if kernel.startswith("clip") else kernel]
    h = hashlib.sha256()
    for f in sorted(files):
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs summarised under profiles/, scaled by the
    copy-kernel calibration; None when absent or taken on other sources."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("{"):
            rec = json.loads(line)
    if not rec or rec.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return rec["hbm_bytes_per_launch"]


def copy_calibration(gib=1.0, reps=5):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps}),
          flush=True)

WORKLOADS = {
    # name: (generator kwargs, tol, default precision)
    "clustered_128": (dict(kind="clustered", n=128, rms=3.0, smooth=1.0, frac=0.2, n_clumps=2000,
                           a=0.5, seed=3), 1e-6, "mixed"),
    "zeldovich_64": (dict(kind="zeldovich", n=64, rms=1.0, smooth=1.0, seed=2), 1e-6, "fp64"),
    "zeldovich_16": (dict(kind="zeldovich", n=16, rms=0.3, smooth=2.0, seed=1), 1e-6, "fp64"),
    # the single large solve (and a quarter-size rehearsal of it)
    "zeldovich_512": (dict(kind="zeldovich", n=512, rms=2.0, smooth=1.0, seed=5), 1e-5, "mixed"),
    "zeldovich_256": (dict(kind="zeldovich", n=256, rms=2.0, smooth=1.0, seed=5), 1e-5, "mixed"),
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


def timed_solves(mak, x_dev, L, tol, precision, steps, warmup, cg_rtol, verbose=0, counting=True):
    import torch
    ctx = mak.Context(0, precision, cg_rtol=cg_rtol, verbose=verbose)
    for w in range(warmup):
        _, _, _, info = ctx.solve(x_dev, L, tol)
        log(f"[bench] warmup {w} {precision}: {info}")
    # HIP events in the timed region bracket the cell-pass kernels only (the
    # roofline's kernel); events around every CG launch would cost ~2 %
    ctx.profile_enable(timing=True, counting=False, cells_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(steps):
        psi, C, D, info = ctx.solve(x_dev, L, tol)
        infos.append(info)
        log(f"[bench] step {k} {precision}: newton={info['newton_iters']} passes={info['cell_passes']} "
            f"cg={info['cg_iters_total']} err={info['final_err']:.2e} t={info['seconds']:.3f}s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    free, total = torch.cuda.mem_get_info()
    prof["_device_mem_used_gb"] = (total - free) / 2 ** 30
    # one more solve outside the timed region with every main kernel timed:
    # the per-kernel breakdown of a solve
    ctx.profile_enable(timing=True, counting=False)
    ctx.solve(x_dev, L, tol)
    bprof = ctx.profile_read()
    prof["_breakdown"] = {k: round(v["total_ms"], 3) for k, v in bprof.items()
                          if not k.startswith("_") and isinstance(v, dict) and "total_ms" in v}
    prof["_spmv"] = bprof.get("spmv")
    cprof = {}
    if counting:
        # counting solve (outside the timed region): work per clip launch
        ctx.profile_enable(timing=True, counting=True)
        ctx.solve(x_dev, L, tol)
        cprof = ctx.profile_read()
    ctx.close()
    return t1 - t0, infos, prof, cprof, (psi, C, D)


def roofline(prof, cprof, workload):
    kern = {k: v for k, v in prof.items() if not k.startswith("_") and k not in ("pcg_solve",)}
    kern = {k: v for k, v in kern.items() if isinstance(v, dict)}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    v = kern[dom]
    avg_ms = v["total_ms"] / max(v["launches"], 1)
    c = cprof.get(dom, v)
    per_launch_flops = c["flops"] / max(c["launches"], 1)
    per_launch_bytes = c["bytes"] / max(c["launches"], 1)
    if dom.startswith("clip") and dom not in cprof:
        # no counting run: the kernel's work is unknown
        out = {"kernel": dom, "bound": "alu", "achieved": None, "peak": PEAK_FP64_VECTOR_TFLOPS,
               "unit": "TFLOP/s", "frac": None, "traffic": None, "avg_launch_ms": avg_ms,
               "launches": v["launches"]}
    elif dom.startswith("clip"):
        # flops: the method's arithmetic only (planes that reach the polytope,
        # vertex tests, new vertices, integrals); the candidate search's
        # counted flops (site scans, ball updates, box tests) are reported
        # beside it, not in `achieved`
        achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
        counters = cprof.get("_counters") or {}
        search_pl = counters.get("search_flops", 0.0) / max(c["launches"], 1)
        out = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
               "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
               "traffic": measured_traffic(dom, workload),
               "avg_launch_ms": avg_ms, "launches": v["launches"],
               "flops_per_launch": per_launch_flops, "bytes_per_launch": per_launch_bytes,
               "cells_per_launch": c["units"] / max(c["launches"], 1),
               "search_flops_per_launch": search_pl,
               "frac_with_search_flops": (per_launch_flops + search_pl) / (avg_ms * 1e-3) / 1e12
                                         / PEAK_FP64_VECTOR_TFLOPS,
               "hbm_GBs_algorithmic": per_launch_bytes / (avg_ms * 1e-3) / 1e9}
    else:
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        out = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
               "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(dom, workload),
               "avg_launch_ms": avg_ms, "launches": v["launches"],
               "bytes_per_launch": per_launch_bytes}
    share = {k: round(kern[k]["total_ms"], 3) for k in kern}
    return out, share


def pass_rates(mak, x_dev, psi, L, precision, reps):
    """Full cell passes (mak_laguerre_cells: volumes, centroids and the CSR
    Hessian) at psi = 0 and at the solved weights: cells/s = N / median pass
    time over `reps` passes after one warm-up, each pass bracketed by device
    synchronisations."""
    import numpy as np
    import torch
    N = x_dev.shape[0]
    ctx = mak.Context(0, precision)
    out = {}
    for name, w in (("psi0", torch.zeros(N, dtype=torch.float64, device=x_dev.device)), ("solved", psi)):
        _, _, info = ctx.laguerre_cells(x_dev, w, L)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.laguerre_cells(x_dev, w, L)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        med = float(np.median(ts))
        out[name] = {"cells_per_s": N / med, "ms_median": med * 1e3, "passes": reps,
                     "nnz": int(info["nnz"]), "max_faces": int(info["max_faces"]),
                     "fp64_rerun_cells": int(info["fp64_rerun_cells"])}
    ctx.close()
    return out


def legendre_leg(mak, x_dev, psi, L, ng, reps, workload):
    """Legendre transform of the solved weights on the ng^3 mesh (node offset
    1/2): phi, cell index and displacement of every node.  HIP-event time of
    the locate kernel over `reps` calls, and of the whole call (site grid
    build included).  Algorithmic bytes per launch: 36 B written per node
    (phi 8, index 4, displacement 24) and 32 B read per site."""
    import torch
    ctx = mak.Context(0)
    ctx.legendre_mesh(x_dev, psi, L, ng, 0.5)
    ctx.profile_enable(timing=True, counting=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.legendre_mesh(x_dev, psi, L, ng, 0.5)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.close()
    v = prof["locate"]
    avg_ms = v["total_ms"] / v["launches"]
    bytes_pl = v["bytes"] / v["launches"]
    achieved = bytes_pl / (avg_ms * 1e-3) / 1e9
    Q = ng ** 3
    return {"mesh": ng, "nodes": Q, "calls": reps,
            "nodes_per_s_kernel": Q / (avg_ms * 1e-3),
            "nodes_per_s_call": Q * reps / (t1 - t0),
            "ms_per_call": (t1 - t0) / reps * 1e3,
            "grid_build_ms": prof["grid_build"]["total_ms"] / prof["grid_build"]["launches"],
            "roofline": {"kernel": "locate", "bound": "hbm", "achieved": achieved,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                         "traffic": measured_traffic("locate", workload),
                         "avg_launch_ms": avg_ms, "launches": v["launches"],
                         "bytes_per_launch": bytes_pl}}


def hbm_roofline(kernel, v, workload):
    """Roofline object of an HBM-bound kernel from its profile entry."""
    avg_ms = v["total_ms"] / v["launches"]
    bytes_pl = v["bytes"] / v["launches"]
    achieved = bytes_pl / (avg_ms * 1e-3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(kernel, workload),
            "avg_launch_ms": avg_ms, "launches": v["launches"], "bytes_per_launch": bytes_pl}


def deposit_and_power(mak, x_dev, psi, L, ng, tau, reps, workload):
    """Zel'dovich deposit of the solved cells at growth amplitude tau (ng^3
    mass elements, cloud in cell onto an ng^3 mesh), then the power spectrum
    of its contrast (CIC window removed).  HIP-event times of the deposit
    kernel, the FFT and the shell binning over `reps` calls each, and of one
    exact deposit of the moved cells."""
    import torch
    ctx = mak.Context(0)
    rho = ctx.za_deposit(x_dev, psi, L, tau, ng, ng, "cic")
    ctx.power_spectrum(rho, L, window=2, contrast=True)
    ctx.profile_enable(timing=True, counting=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rho = ctx.za_deposit(x_dev, psi, L, tau, ng, ng, "cic")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        k, P, m = ctx.power_spectrum(rho, L, window=2, contrast=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # the exact deposit of the moved cells (a float64 cell pass with faces,
    # then each cell clipped against the voxels it reaches): one warm call
    ctx.za_deposit_cells(x_dev, psi, L, tau, ng)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rho_x = ctx.za_deposit_cells(x_dev, psi, L, tau, ng)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.close()
    dep = prof["deposit"]
    cdep = prof["cells_deposit"]
    rho_c = rho.cpu()
    N = x_dev.shape[0]
    cells_kernel_ms = cdep["total_ms"] / cdep["launches"]
    return {
        "deposit_cells": {"tau": tau, "cells": N, "mesh": ng, "ms_per_call": (t4 - t3) * 1e3,
                          "kernel_ms": cells_kernel_ms, "cells_per_s_kernel": N / (cells_kernel_ms * 1e-3),
                          "mass_rel_err": float(rho_x.sum().item() / ng ** 3 - 1.0)},
        "deposit": {"tau": tau, "elements": ng ** 3, "mesh": ng, "scheme": "cic",
                    "ms_per_call": (t1 - t0) / reps * 1e3,
                    "elements_per_s_kernel": ng ** 3 / (dep["total_ms"] / dep["launches"] * 1e-3),
                    "density_min": float(rho_c.min()), "density_max": float(rho_c.max()),
                    "roofline": hbm_roofline("deposit", dep, workload)},
        "power_spectrum": {"mesh": ng, "shells": int(P.numel()), "window": "cic", "contrast": True,
                           "ms_per_call": (t2 - t1) / reps * 1e3,
                           "fft_ms": prof["fft"]["total_ms"] / prof["fft"]["launches"],
                           "P_first_shells": [float(v) for v in P[:4].cpu()],
                           "roofline": hbm_roofline("shell_bin", prof["shell_bin"], workload)},
    }


def compare_paths(a, b, L, N):
    """rms / max differences between the two precision paths' solutions, in
    grid units (spacing L / N^(1/3))."""
    import numpy as np
    D = L / N ** (1.0 / 3.0)
    pa, ca, da = (t.cpu().numpy() for t in a)
    pb, cb, db = (t.cpu().numpy() for t in b)
    dc = ca - cb
    dc -= L * np.round(dc / L)
    dd = da - db
    return {"centroid_rms_grid": float(np.sqrt(np.mean(np.sum(dc * dc, 1))) / D),
            "centroid_max_grid": float(np.abs(dc).max() / D),
            "disp_rms_grid": float(np.sqrt(np.mean(np.sum(dd * dd, 1))) / D),
            "psi_rms_over_D2": float(np.sqrt(np.mean((pa - pa.mean() - pb + pb.mean()) ** 2)) / D ** 2)}


def accuracy_vs_oracle(mak, x, out, L, sample=64):
    """Mixed-precision cell pass at its converged weights against the float64
    oracle on sampled cells: max relative volume error, centroid error in
    grid units, and the oracle's own volume error (solve certificate)."""
    import numpy as np
    import torch

    import oracle
    psi = out[0]
    N = x.shape[0]
    D = L / N ** (1.0 / 3.0)
    ctx = mak.Context(0, "mixed")
    V, C, info = ctx.laguerre_cells(torch.from_numpy(x).cuda(), psi, L)
    F = {k: v.cpu().numpy() for k, v in ctx.faces().items()}
    ctx.close()
    V = V.cpu().numpy()
    C = C.cpu().numpy()
    idx = np.random.default_rng(7).choice(N, sample, replace=False)
    r = oracle.cells(x, psi.cpu().numpy(), L, idx=idx, threads=min(os.cpu_count() or 1, 16))
    uo = r["M"] / r["V"][:, None]
    co = np.mod(x[idx] + uo, L)
    dc = C[idx] - co
    dc -= L * np.round(dc / L)
    m = L ** 3 / N
    # adjacency: faces (j, image) of the sampled cells reported by one side
    # only, split at the mixed path's area threshold tau_A = 1e-6 spacing^2
    tau_a = 1e-6 * D * D
    above = below = matched = 0
    for k, i in enumerate(idx):
        fo = {key: a for key, (a, _d) in oracle.cell_faces_dict(r, k).items()}
        fg = {}
        for f in range(F["face_ptr"][i], F["face_ptr"][i + 1]):
            fg[(int(F["face_j"][f]),) + tuple(int(t) for t in F["face_shift"][f])] = float(F["face_area"][f])
        for key in set(fo) ^ set(fg):
            if fo.get(key, fg.get(key)) >= tau_a:
                above += 1
            else:
                below += 1
        matched += len(set(fo) & set(fg))
    return {"sample_cells": sample,
            "max_rel_volume_err": float(np.max(np.abs(V[idx] - r["V"]) / r["V"])),
            "centroid_rms_grid": float(np.sqrt(np.mean(np.sum(dc * dc, 1))) / D),
            "disp_rms_grid": float(np.sqrt(np.mean(np.sum(dc * dc, 1))) / D),
            "oracle_max_rel_volume_err_vs_m": float(np.max(np.abs(r["V"] - m)) / m),
            "faces_matched": matched, "adjacency_diff_above_tau": above,
            "adjacency_diff_below_tau": below, "tau_A_over_spacing2": 1e-6,
            "fp64_rerun_cells_in_pass": int(info["fp64_rerun_cells"])}


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
    # one thread, on an eighth of the time
    m1 = int(max(4, min(N, seconds / 8 / max(per_cell * threads, 1e-9))))
    idx1 = rng.choice(N, m1, replace=False)
    t1 = time.perf_counter()
    oracle.cells(x, psi, L, idx=idx1, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": m / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} random cells of the same {N}-site input at psi=0 "
                      f"(one cell pass, {dt:.1f} s)",
            "single_thread_cells_per_s": m1 / dt1, "single_thread_sample_cells": m1}


def oracle_small_timings(threads):
    """The oracle on the small configurations it runs whole: one cell pass at
    16^3 and at 32^3 (psi = 0), and the full damped-Newton solve of the
    16^3 input (dense Newton steps) to 1e-6."""
    import numpy as np

    import oracle
    import workloads
    out = {"threads": threads}
    for n in (16, 32):
        x = workloads.zeldovich(n, rms=0.3 if n == 16 else 1.0, smooth=2.0 if n == 16 else 1.0,
                                seed=1 if n == 16 else 2)
        t0 = time.perf_counter()
        oracle.cells(x, np.zeros(len(x)), 1.0, threads=threads)
        dt = time.perf_counter() - t0
        out[f"pass_{n}"] = {"N": len(x), "seconds": dt, "cells_per_s": len(x) / dt}
    x = workloads.zeldovich(16, rms=0.3, smooth=2.0, seed=1)
    t0 = time.perf_counter()
    r = oracle.solve(x, 1.0, 1e-6, threads=threads)
    out["solve_16"] = {"N": len(x), "seconds": time.perf_counter() - t0,
                       "newton_iters": int(r["newton_iters"]), "final_err": float(r["err"])}
    return out


def serving(mak, count, slots, budget_gb, precision, tol, cg_rtol, window_us=0, seed=1000):
    """Continuous-batching serving: requests of the serving mix (lattice side
    log-uniform in [32, 128], rms 0.5..3 spacings) arrive as a Poisson process
    at 0.8 x the closed-loop capacity (the whole mix submitted at once, which
    also warms the workspaces); latency is submit -> done."""
    import numpy as np
    import torch

    import workloads
    reqs = workloads.serving_requests(count, seed=seed)
    log(f"[bench] serving: generating {count} inputs ...")
    xs = [torch.from_numpy(workloads.zeldovich(r["n"], rms=r["rms"], smooth=r["smooth"],
                                               seed=r["seed"])).cuda() for r in reqs]
    torch.cuda.synchronize()
    budget = int(budget_gb * (1 << 30))
    live0, _ = mak.device_bytes(reset_peak=True)
    srv = mak.Server(0, precision, mem_budget=budget, max_slots=slots, cg_rtol=cg_rtol,
                     batch_window_us=window_us)
    # closed-loop capacity: the whole mix submitted at once
    t0 = time.perf_counter()
    rs = [srv.submit(x, 1.0, tol) for x in xs]
    for r in rs:
        r.wait()
    cap = len(xs) / (time.perf_counter() - t0)
    lam = 0.8 * cap
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, len(xs)))
    log(f"[bench] serving: capacity {cap:.2f} req/s, arrival rate {lam:.2f} req/s")
    t0 = time.perf_counter()
    sub = []
    for x, ta in zip(xs, arrivals):
        dt = t0 + ta - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        sub.append(srv.submit(x, 1.0, tol))
    for r in sub:
        r.wait()
    lat = np.array([r.times[2] - r.times[0] for r in sub])
    span = max(r.times[2] for r in sub) - min(r.times[0] for r in sub)
    st = srv.stats()
    _, peak = mak.device_bytes()
    srv.close()
    ns = np.array([r["n"] ** 3 for r in reqs])
    return {"requests": len(sub), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "requests_per_s": len(sub) / span,
            "arrival_rate_per_s": lam, "closed_loop_capacity_per_s": cap, "slots": slots,
            "mem_budget_gb": budget_gb, "peak_used_gb": st["peak_used_bytes"] / 2 ** 30,
            "peak_device_gb_measured": (peak - live0) / 2 ** 30,
            "workspace_releases": st["releases"],
            "peak_active": st["peak_active"], "admitted_while_busy": st["admitted_while_busy"],
            "cell_passes_per_shared_launch": st["batched_passes"] / max(st["pass_batches"], 1),
            "max_passes_in_one_launch": st["max_batch"],
            "N_min": int(ns.min()), "N_median": int(np.median(ns)), "N_max": int(ns.max()),
            "batch_window_us": window_us, "precision": precision, "tol": tol}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="clustered_128", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--compare", default="auto", choices=["auto", "fp64", "mixed", "none"],
                    help="also time another precision path (auto: the other one)")
    ap.add_argument("--cg-rtol", type=float, default=1e-3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", type=int, nargs="?", const=1, default=0,
                    help="solver log on stderr: 1 per Newton iteration, 2 also per line-search trial")
    ap.add_argument("--no-counting", action="store_true",
                    help="skip the extra solve with the clip kernel's work counters")
    ap.add_argument("--pass-reps", type=int, default=10,
                    help="timed full cell passes at psi = 0 and at the solved weights (0 = skip)")
    ap.add_argument("--oracle-sample", type=int, default=64,
                    help="cells of the mixed path checked against the oracle")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving leg (0 = skip)")
    ap.add_argument("--legendre-reps", type=int, default=5,
                    help="calls of the Legendre transform, the Zel'dovich deposit and the power "
                         "spectrum on the mesh at the solved weights (0 = skip)")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-window-us", type=int, default=2000,
                    help="batch window of the serving leg's pass batcher (microseconds)")
    ap.add_argument("--serving-budget-gb", type=float, default=6.0,
                    help="memory budget of the serving leg (the largest request needs ~2.4 GB, "
                         "so the slots' workspaces bind it)")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the mixed path's sampled check against the oracle")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the domain "
              "decomposition over several GPUs is not implemented.", file=sys.stderr)
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

    secs, infos, prof, cprof, out = timed_solves(mak, x_dev, L, tol, precision, args.steps,
                                                 args.warmup, args.cg_rtol, int(args.verbose),
                                                 counting=not args.no_counting)
    # cells of complete passes only: a line-search trial abandoned at its
    # first cell below eps0 counts as no cells
    passes = sum(i["cell_passes"] - i["abandoned_trials"] for i in infos)
    value = N * passes / secs
    rl, _ = roofline(prof, cprof, args.workload)
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
                  "abandoned_trials": infos[-1]["abandoned_trials"],
                  "cg_iters": infos[-1]["cg_iters_total"], "final_err": infos[-1]["final_err"]},
        "kernel_ms_one_solve": prof.get("_breakdown"),
        # the second kernel of the solve (CG), against the HBM roofline
        "spmv_roofline": hbm_roofline("spmv", prof["_spmv"], args.workload) if prof.get("_spmv") else None,
        "device_mem_used_gb": prof.get("_device_mem_used_gb"),
        "work_counters_per_solve": cprof.get("_counters"),
        "roofline": rl,
    }
    other = args.compare
    if other == "auto":
        other = "fp64" if precision == "mixed" else "mixed"
    if other not in ("none", precision):
        s2, inf2, p2, c2, out2 = timed_solves(mak, x_dev, L, tol, other, max(1, args.steps), 0,
                                              args.cg_rtol)
        res[other] = {"cells_per_s": N * sum(i["cell_passes"] - i["abandoned_trials"] for i in inf2) / s2,
                      "ms_per_solve": s2 / len(inf2) * 1e3,
                      "newton_iters": inf2[-1]["newton_iters"], "final_err": inf2[-1]["final_err"],
                      "fp64_rerun_cells": inf2[-1]["fp64_rerun_cells"]}
        res["paths_agreement"] = compare_paths(out, out2, L, N)
    if (precision == "mixed" or other == "mixed") and not args.no_oracle_check:
        res["mixed_vs_oracle"] = accuracy_vs_oracle(mak, x, out if precision == "mixed" else out2, L,
                                                    sample=args.oracle_sample)
    if args.pass_reps > 0:
        log("[bench] full cell passes at psi = 0 and at the solved weights ...")
        res["cell_pass"] = {precision: pass_rates(mak, x_dev, out[0], L, precision, args.pass_reps)}
        if other not in ("none", precision):
            res["cell_pass"][other] = pass_rates(mak, x_dev, out2[0], L, other, args.pass_reps)
    if args.legendre_reps > 0:
        ng = round(N ** (1.0 / 3.0))
        log(f"[bench] Legendre transform on the {ng}^3 mesh ...")
        res["legendre"] = legendre_leg(mak, x_dev, out[0], L, ng, args.legendre_reps, args.workload)
    if args.legendre_reps > 0:
        ng = round(N ** (1.0 / 3.0))
        log(f"[bench] Zel'dovich deposit and power spectrum on the {ng}^3 mesh ...")
        res.update(deposit_and_power(mak, x_dev, out[0], L, ng, 0.5, args.legendre_reps, args.workload))
    if args.serving_requests > 0:
        res["serving"] = serving(mak, args.serving_requests, args.serving_slots,
                                 args.serving_budget_gb, precision, tol, args.cg_rtol,
                                 args.serving_window_us)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(x, L, args.cpu_seconds)
        res["cpu_baseline"]["small_configs"] = oracle_small_timings(res["cpu_baseline"]["cores"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
