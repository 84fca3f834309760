"""Serving (continuous batching of solves) through the C-ABI server.

Each served result is the same bits as a solo solve of the same input, and is
certified by the oracle: the oracle's cells at the served weights meet the
stop tolerance (Eq. SDK gradient m - V), the served centroids are the
oracle's, and a cell pass at the served weights on the served path's
precision has the oracle's adjacency, volumes and centroids."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import compare_cells, gpu_faces

pytestmark = pytest.mark.gpu

TOL = 1e-8


def _inputs():
    reqs = [(8, 0.5, 11), (12, 1.0, 12), (16, 0.4, 13), (10, 2.0, 14), (20, 0.8, 15)]
    return [workloads.zeldovich(n, rms=rms, smooth=1.0, seed=s) for n, rms, s in reqs]


def _certify(ctx, x, psi, C, D):
    """Oracle certificate of one served result (numpy arrays, original
    order); ctx runs the cell pass at the served weights."""
    import torch
    N = len(x)
    sp = 1.0 / N ** (1.0 / 3.0)
    res = oracle.cells(x, psi, 1.0)
    err = np.max(np.abs(res["V"] * N - 1.0))
    assert err <= TOL * 1.01, f"oracle volumes at the served psi: {err:.3e}"
    u = res["M"] / res["V"][:, None]
    dc = C - np.mod(x + u, 1.0)
    dc -= np.round(dc)
    assert np.abs(dc).max() <= 1e-10 * sp
    assert np.abs(D + u).max() <= 1e-10 * sp
    V, Cg, _ = ctx.laguerre_cells(torch.from_numpy(x).cuda(), torch.from_numpy(psi).cuda(), 1.0)
    rep = compare_cells(x, psi, 1.0, V.cpu().numpy(), Cg.cpu().numpy(), gpu_faces(ctx), res=res)
    return err, rep


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_same_alone_and_in_the_mix(precision):
    import torch

    import paper_2110_08868_amd as mak
    xs = _inputs()
    ctx = mak.Context(0, precision, cg_rtol=1e-6)
    solo = [tuple(t.cpu().numpy() for t in ctx.solve(torch.from_numpy(x), 1.0, TOL)[:3]) for x in xs]
    # a batch window long enough that the first passes of the admitted
    # requests always meet (the batch fires once every solve in flight has
    # posted)
    srv = mak.Server(0, precision, max_slots=3, cg_rtol=1e-6, batch_window_us=200000)
    reqs = [srv.submit(torch.from_numpy(x), 1.0, TOL) for x in xs]
    for x, r, (p0, c0, d0) in zip(xs, reqs, solo):
        psi, C, D, info = r.wait()
        assert info["final_err"] <= TOL
        psi, C, D = psi.cpu().numpy(), C.cpu().numpy(), D.cpu().numpy()
        assert np.array_equal(psi, p0)
        assert np.array_equal(C, c0)
        assert np.array_equal(D, d0)
        err, rep = _certify(ctx, x, psi, C, D)
        print(f"  {precision} N={len(x)} oracle err {err:.2e} {rep}", flush=True)
    ctx.close()
    st = srv.stats()
    print("  server stats", st, flush=True)
    assert st["completed"] == len(xs) and st["peak_active"] >= 2
    # the cell passes of concurrent requests shared launches
    assert st["max_batch"] >= 2 and st["batched_passes"] > st["pass_batches"]
    srv.close()


def test_admission_by_memory():
    """The budget holds one big workspace and half a small one: the two big
    requests never run (or sit) together, idle workspaces stay charged, and
    what the library really allocates stays within the budget."""
    import torch

    import paper_2110_08868_amd as mak
    small = workloads.zeldovich(8, rms=0.5, smooth=1.0, seed=3)
    big = workloads.zeldovich(24, rms=0.5, smooth=1.0, seed=4)
    est_small = mak.memory_estimate(len(small))
    est_big = mak.memory_estimate(len(big))
    budget = est_big + est_small // 2
    live0, _ = mak.device_bytes(reset_peak=True)
    srv = mak.Server(0, mem_budget=budget, max_slots=4)
    huge = workloads.zeldovich(48, rms=0.5, smooth=1.0, seed=5)
    assert mak.memory_estimate(len(huge)) > budget
    with pytest.raises(mak.MakError) as e:
        srv.submit(torch.from_numpy(huge), 1.0)
    assert e.value.name == "MAK_ENOMEM"
    rs = [srv.submit(torch.from_numpy(big), 1.0, 1e-6), srv.submit(torch.from_numpy(small), 1.0, 1e-6),
          srv.submit(torch.from_numpy(big), 1.0, 1e-6)]
    for r in rs:
        r.wait()
    st = srv.stats()
    live, peak = mak.device_bytes()
    print(f"  stats {st}; library device bytes peak {peak - live0} live {live - live0} "
          f"budget {budget}", flush=True)
    assert st["peak_used_bytes"] <= st["budget_bytes"]
    # measured: what the library allocated beyond what it held before
    assert peak - live0 <= budget
    # the idle big workspace is still charged after the last request
    assert st["used_bytes"] >= est_big
    # the second big request started after the first ended
    assert rs[2].times[1] >= rs[0].times[2] - 1e-3
    srv.close()
    live1, _ = mak.device_bytes()
    assert live1 == live0


def test_admitted_while_busy():
    import torch

    import paper_2110_08868_amd as mak
    srv = mak.Server(0, max_slots=2)
    big = srv.submit(torch.from_numpy(workloads.zeldovich(40, rms=1.5, smooth=1.0, seed=6)), 1.0, 1e-7)
    smalls = [srv.submit(torch.from_numpy(workloads.zeldovich(8, rms=0.5, smooth=1.0, seed=7 + k)),
                         1.0, 1e-7) for k in range(4)]
    for s in smalls:
        s.wait()
    big.wait()
    # the small requests were served while the big one ran
    assert min(s.times[2] for s in smalls) < big.times[2]
    assert srv.stats()["admitted_while_busy"] >= 1
    srv.close()
