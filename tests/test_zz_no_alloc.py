"""mak_legendre_noalloc (the Legendre transform and point location with the
library's workspace in its static device array) against mak_legendre, the
entry point it shares its kernels with: the same bits on two calls in a row,
the second with a smaller input (the array keeps the first call's contents),
and no device memory allocated by the library during either call."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _case(n, nq, seed):
    x = workloads.zeldovich(n, rms=1.0, smooth=1.0, seed=seed)
    rng = np.random.default_rng(seed)
    psi = rng.uniform(-1, 1, len(x)) * 0.3 / n ** 2
    q = rng.uniform(-0.5, 1.5, (nq, 3))
    return x, psi, q


def test_no_alloc_matches_legendre():
    import torch

    import paper_2110_08868_amd as mak
    ctx = mak.Context(0)
    try:
        for n, nq, seed in ((40, 30000, 91), (12, 700, 92)):
            print(f"case N={n ** 3} Q={nq} seed={seed}", flush=True)
            x, psi, q = _case(n, nq, seed)
            xd = torch.from_numpy(x).cuda()
            pd = torch.from_numpy(psi).cuda()
            qd = torch.from_numpy(q).cuda()
            ref = [t.cpu().numpy() for t in ctx.legendre(xd, pd, 1.0, qd)]
            out = (torch.empty(nq, dtype=torch.float64, device="cuda"),
                   torch.empty(nq, dtype=torch.int32, device="cuda"),
                   torch.empty((nq, 3), dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            live0, _ = mak.device_bytes(reset_peak=True)
            got = ctx.legendre_noalloc(xd, pd, 1.0, qd, out=out)
            torch.cuda.synchronize()
            live1, peak = mak.device_bytes()
            assert live1 == live0 and peak == live0, "the library allocated device memory"
            got = [t.cpu().numpy() for t in got]
            for a, b in zip(got, ref):
                assert np.array_equal(a, b)
            # the located cell attains the minimum of the power distances
            d = x[got[1]] - np.mod(q, 1.0)
            d -= np.round(d)
            v = 0.5 * np.sum(d * d, axis=1) - psi[got[1]]
            assert np.abs(v - got[0]).max() <= 1e-13
    finally:
        ctx.close()


def test_no_alloc_rejects_what_does_not_fit():
    import torch

    import paper_2110_08868_amd as mak
    ctx = mak.Context(0)
    try:
        x = np.random.default_rng(5).uniform(0, 1, (1_000_000, 3))
        q = np.random.default_rng(6).uniform(0, 1, (10, 3))
        with pytest.raises(mak.MakError) as e:
            ctx.legendre_noalloc(torch.from_numpy(x).cuda(), None, 1.0, torch.from_numpy(q).cuda())
        assert e.value.name == "MAK_EINVAL" and "workspace" in e.value.message
        # the context still works after the refusal
        x, psi, qq = _case(6, 50, 93)
        ctx.legendre_noalloc(torch.from_numpy(x).cuda(), torch.from_numpy(psi).cuda(), 1.0,
                             torch.from_numpy(qq).cuda())
    finally:
        ctx.close()
