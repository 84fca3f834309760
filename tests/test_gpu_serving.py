"""Serving (continuous batching of solves) through the C-ABI server."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _inputs():
    reqs = [(8, 0.5, 11), (12, 1.0, 12), (16, 0.4, 13), (10, 2.0, 14), (20, 0.8, 15)]
    return [workloads.zeldovich(n, rms=rms, smooth=1.0, seed=s) for n, rms, s in reqs]


def test_same_alone_and_in_the_mix():
    import torch

    import paper_2110_08868_amd as mak
    xs = _inputs()
    ctx = mak.Context(0, cg_rtol=1e-6)
    solo = [tuple(t.cpu().numpy() for t in ctx.solve(torch.from_numpy(x), 1.0, 1e-8)[:3]) for x in xs]
    ctx.close()
    # a batch window long enough that the first passes of the admitted
    # requests always meet (the batch fires once every solve in flight has
    # posted)
    srv = mak.Server(0, max_slots=3, cg_rtol=1e-6, batch_window_us=200000)
    reqs = [srv.submit(torch.from_numpy(x), 1.0, 1e-8) for x in xs]
    for r, (p0, c0, d0) in zip(reqs, solo):
        psi, C, D, info = r.wait()
        assert info["final_err"] <= 1e-8
        assert np.array_equal(psi.cpu().numpy(), p0)
        assert np.array_equal(C.cpu().numpy(), c0)
        assert np.array_equal(D.cpu().numpy(), d0)
    st = srv.stats()
    print("  server stats", st, flush=True)
    assert st["completed"] == len(xs) and st["peak_active"] >= 2
    # the cell passes of concurrent requests shared launches
    assert st["max_batch"] >= 2 and st["batched_passes"] > st["pass_batches"]
    srv.close()


def test_admission_by_memory():
    import torch

    import paper_2110_08868_amd as mak
    small = workloads.zeldovich(8, rms=0.5, smooth=1.0, seed=3)
    big = workloads.zeldovich(24, rms=0.5, smooth=1.0, seed=4)
    est_small = mak.memory_estimate(len(small))
    est_big = mak.memory_estimate(len(big))
    # the budget holds one big request, or the big one is rejected outright
    budget = est_big + est_small // 2
    srv = mak.Server(0, mem_budget=budget, max_slots=4)
    huge = workloads.zeldovich(48, rms=0.5, smooth=1.0, seed=5)
    assert mak.memory_estimate(len(huge)) > budget
    with pytest.raises(mak.MakError) as e:
        srv.submit(torch.from_numpy(huge), 1.0)
    assert e.value.name == "MAK_ENOMEM"
    r1 = srv.submit(torch.from_numpy(big), 1.0, 1e-6)
    r2 = srv.submit(torch.from_numpy(big), 1.0, 1e-6)
    r1.wait()
    r2.wait()
    st = srv.stats()
    assert st["peak_used_bytes"] <= st["budget_bytes"]
    # two big requests never ran together
    assert r2.times[1] >= r1.times[2] - 1e-3
    srv.close()


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
