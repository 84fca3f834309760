"""Comparison of the HIP cell pass with the CPU oracle (shared by GPU tests).

Tolerances (FP64 path): volumes and centroids to 1e-10 relative to the cell
volume / the mean site spacing; faces compared above the area threshold
tau = 1e-12 spacing^2 (faces that straddle the threshold, i.e. below
100 tau on the side that reports them, are counted, not failed); matched face
areas to 1e-10 relative to max(area, 1e-3 spacing^2): a thin sliver face has
an absolute rounding floor of about 1e-16 spacing^2 times its aspect ratio on
both sides, so its relative error is not bounded by 1e-10; Hessian entries to
1e-9 of the largest entry.
"""
from __future__ import annotations

import numpy as np

import oracle


def spacing(N, L):
    return L / N ** (1.0 / 3.0)


def gpu_faces(ctx):
    f = ctx.faces()
    return {k: v.cpu().numpy() for k, v in f.items()}


def face_dict_gpu(F, i, tau):
    out = {}
    for f in range(F["face_ptr"][i], F["face_ptr"][i + 1]):
        a = float(F["face_area"][f])
        if a > tau:
            out[(int(F["face_j"][f]),) + tuple(int(s) for s in F["face_shift"][f])] = a
    return out


def compare_cells(x, psi, L, V, C, F, res=None, idx=None, vol_rel=1e-10, cen_rel=1e-10,
                  area_rel=1e-10):
    """Compare GPU volumes V, centroids C and faces F (numpy, original order)
    with the oracle on cells `idx` (all by default).  Returns a report dict
    and raises AssertionError on a parity failure."""
    N = x.shape[0]
    D = spacing(N, L)
    tau = 1e-12 * D * D
    if res is None:
        res = oracle.cells(x, psi, L, idx=idx)
    idx = res["idx"]
    vm = L ** 3 / N
    Vo = res["V"]
    dV = np.abs(V[idx] - Vo)
    assert np.all(dV <= vol_rel * np.maximum(Vo, 1e-3 * vm)), \
        f"volume mismatch: max rel {np.max(dV / np.maximum(Vo, 1e-3 * vm)):.3e}"
    uo = np.where(Vo[:, None] > 0, res["M"] / np.where(Vo > 0, Vo, 1)[:, None], 0.0)
    co = np.mod(x[idx] + uo, L)
    dc = C[idx] - co
    dc -= L * np.round(dc / L)
    cerr = np.abs(dc).max() / D if len(idx) else 0.0
    assert cerr <= cen_rel, f"centroid mismatch {cerr:.3e} spacings"
    straddle = 0
    aerr = 0.0
    for k, i in enumerate(idx):
        fo = {key: a for key, (a, _d) in oracle.cell_faces_dict(res, k, min_area=tau).items()}
        fg = face_dict_gpu(F, i, tau)
        for key in set(fo) ^ set(fg):
            a = fo.get(key, fg.get(key))
            assert a < 100 * tau, f"cell {i}: face {key} area {a:.3e} on one side only"
            straddle += 1
        for key in set(fo) & set(fg):
            e = abs(fo[key] - fg[key]) / max(fo[key], D * D * 1e-3)
            aerr = max(aerr, e)
    assert aerr <= area_rel, f"face area mismatch {aerr:.3e}"
    return {"max_vol_rel": float(np.max(dV / np.maximum(Vo, 1e-3 * vm))) if len(idx) else 0.0,
            "max_cen_spacings": float(cerr), "max_area_rel": aerr, "straddling_faces": straddle}


def csr_to_dense(rp, col, val, N):
    J = np.zeros((N, N))
    for i in range(N):
        for k in range(rp[i], rp[i + 1]):
            J[i, col[k]] += val[k]
    return J
