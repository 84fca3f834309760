"""GPU power spectrum of a mesh field (mak_power_spectrum) against the numpy
FFT oracle: mode counts bit-exact, mean |k| and mean P to rounding."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2110_08868_amd as mak
    c = mak.Context(0)
    yield c
    c.close()


def gpk(ctx, f, L, **kw):
    import torch
    k, P, m = ctx.power_spectrum(torch.from_numpy(f), L, **kw)
    return k.cpu().numpy(), P.cpu().numpy(), m.cpu().numpy()


def field(ng, seed, positive=False):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(ng, ng, ng))
    return np.exp(0.5 * f) if positive else f


def check(ctx, f, L, nbins=None, window=0, contrast=False):
    k, P, m = gpk(ctx, f, L, nbins=nbins, window=window, contrast=contrast)
    rk, rP, rm = oracle.power_spectrum(f, L, nbins=nbins, window=window, contrast=contrast)
    assert np.array_equal(m, rm)
    ok = rm > 0
    assert np.all(np.isnan(P[~ok])) and np.all(np.isnan(k[~ok]))
    # a shell sums m terms in another order on each side: rounding grows
    # like sqrt(m) ulps
    tol = 1e-14 + 2e-15 * np.sqrt(rm[ok])
    eP = np.abs(P[ok] - rP[ok]) / np.abs(rP[ok])
    ek = np.abs(k[ok] - rk[ok]) / rk[ok]
    print(f"  ng={f.shape[0]} nbins={len(m)} window={window} contrast={contrast}: "
          f"max rel dP={eP.max():.2e} dk={ek.max():.2e}", flush=True)
    assert np.all(eP <= tol) and np.all(ek <= tol)
    return k, P, m


@pytest.mark.parametrize("ng,window,contrast,nbins", [
    (16, 0, False, None), (12, 2, True, 20), (9, 1, False, None), (33, 3, False, None),
    (2, 0, False, 2), (64, 2, True, None), (10, 0, False, 3)])
def test_vs_oracle(ctx, ng, window, contrast, nbins):
    check(ctx, field(ng, 60 + ng, positive=contrast), 2.5, nbins=nbins, window=window, contrast=contrast)


def test_plane_wave_closed_form(ctx):
    ng, L, A = 32, 1.0, 0.4
    t = np.arange(ng) * (L / ng)
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    n0 = np.array([3, 4, 0])
    f = A * np.cos(2 * np.pi * (n0[0] * X + n0[1] * Y + n0[2] * Z) / L + 0.2)
    k, P, m = gpk(ctx, f, L)
    j0 = 5
    assert P[j0 - 1] * m[j0 - 1] == pytest.approx(2 * A * A * L ** 3 / 4, rel=1e-12)
    other = np.delete(P * m, j0 - 1)
    assert np.max(np.abs(other)) <= 1e-25


def test_deterministic_and_plan_changes(ctx):
    a = field(24, 71)
    b = field(20, 72)
    r1 = gpk(ctx, a, 1.0, window=2)
    gpk(ctx, b, 1.0)  # another mesh size replaces the plan
    r2 = gpk(ctx, a, 1.0, window=2)
    for u, v in zip(r1, r2):
        assert np.array_equal(u, v, equal_nan=True)


@pytest.mark.parametrize("ng", [128, 256])
def test_full_size(ctx, ng):
    """The mesh sizes of the deposited fields (128^3: one node per site of
    the 128^3 inputs), every shell against the oracle."""
    f = field(ng, 80 + ng, positive=True)
    check(ctx, f, 1.0, window=2, contrast=True)


def test_errors(ctx):
    import torch
    import paper_2110_08868_amd as mak
    f = torch.from_numpy(field(8, 90))
    for kw in (dict(nbins=0), dict(window=4), dict(nbins=4096)):
        with pytest.raises(mak.MakError) as e:
            ctx.power_spectrum(f, 1.0, **kw)
        assert e.value.name == "MAK_EINVAL"
    z = torch.zeros((8, 8, 8), dtype=torch.float64)
    with pytest.raises(mak.MakError) as e:
        ctx.power_spectrum(z, 1.0, contrast=True)
    assert e.value.name == "MAK_EINVAL"
    with pytest.raises(ValueError):
        ctx.power_spectrum(torch.zeros((8, 8, 4), dtype=torch.float64), 1.0)
    gpk(ctx, field(8, 91), 1.0)
