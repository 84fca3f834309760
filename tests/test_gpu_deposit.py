"""GPU Zel'dovich advection and Eulerian deposit (mak_za_deposit) against the
oracle.

The GPU sums masses in 64-bit fixed point: U = 2^(62 - ceil(log2 n_lag^3))
units per element (at most 2^52), each cloud-in-cell weight rounded to
units (error <= 1/2 unit) and the remainder (<= 7/2 units) on the heaviest
node.  A node's deposit therefore differs from the float64 sum by at most
4 units per element that reaches it; with every element reaching a node
that is 4 n_lag^3 / U units of mass (L / n_lag)^3 / U each, i.e. a density
error below 4 ng^3 / U (L = 1), plus float64 rounding."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2110_08868_amd as mak
    c = mak.Context(0)
    yield c
    c.close()


def units(n_lag):
    bits = int(np.ceil(np.log2(n_lag ** 3))) if n_lag > 1 else 0
    return 2.0 ** min(62 - bits, 52)


def gdep(ctx, x, psi, L, tau, n_lag, ng, scheme, off=0.5):
    import torch
    r = ctx.za_deposit(torch.from_numpy(x), None if psi is None else torch.from_numpy(psi), L, tau,
                       n_lag, ng, scheme, off)
    return r.cpu().numpy()


@pytest.mark.parametrize("tau,scheme,n_lag,ng", [
    (0.35, "cic", 12, 8), (0.9, "ngp", 10, 6), (1.0, "cic", 9, 7), (0.0, "ngp", 8, 8),
    (0.6, "cic", 16, 12), (0.5, "ngp", 5, 1)])
def test_vs_oracle(ctx, tau, scheme, n_lag, ng):
    n = 4
    x = workloads.zeldovich(n, rms=0.6, smooth=1.0, seed=71)
    rng = np.random.default_rng(71)
    psi = rng.uniform(-1, 1, len(x)) * 0.03 / n ** 2
    r = gdep(ctx, x, psi, 1.0, tau, n_lag, ng, scheme)
    o = oracle.za_deposit(x, psi, 1.0, tau, n_lag, ng, scheme=scheme)
    tol = 4.0 * ng ** 3 / units(n_lag) + 1e-12
    err = np.abs(r - o).max()
    print(f"  tau={tau} {scheme} n_lag={n_lag} ng={ng}: max |drho|={err:.2e} (tol {tol:.1e})", flush=True)
    assert err <= tol
    assert r.sum() / ng ** 3 == pytest.approx(1.0, rel=1e-14)


def test_clustered_box_size_and_offsets(ctx):
    L = 3.0
    x = workloads.clustered(6, L=L, seed=73)
    rng = np.random.default_rng(73)
    psi = rng.uniform(-1, 1, len(x)) * 0.02 * (L / 6) ** 2
    for tau, sch, off in ((0.5, "cic", 0.0), (0.75, "ngp", 0.3)):
        r = gdep(ctx, x, psi, L, tau, 11, 9, sch, off)
        o = oracle.za_deposit(x, psi, L, tau, 11, 9, scheme=sch, lag_offset=off)
        assert np.abs(r - o).max() <= 4.0 * 9 ** 3 / units(11) + 1e-12


def test_layered_separable(ctx):
    """The separable layered case of the oracle's pins, on the GPU."""
    from tests.closed_forms import layered_ot_psi
    rng = np.random.default_rng(61)
    L, nl, ny = 1.0, 3, 2
    X = np.sort(rng.uniform(0, L, nl))
    w = rng.uniform(0.6, 1.4, nl)
    w *= L / w.sum()
    psi_l, _ = layered_ot_psi(X, L, widths=w)
    x = workloads.layered(X, ny, ny, L)
    psi = np.repeat(psi_l, ny * ny)
    r = gdep(ctx, x, psi, L, 0.4, 24, 8, "ngp")
    o = oracle.za_deposit(x, psi, L, 0.4, 24, 8, scheme="ngp")
    assert np.abs(r - o).max() <= 4.0 * 8 ** 3 / units(24) + 1e-12


def test_deterministic(ctx):
    x = workloads.clustered(8, seed=75)
    a = gdep(ctx, x, None, 1.0, 0.7, 20, 16, "cic")
    b = gdep(ctx, x, None, 1.0, 0.7, 20, 16, "cic")
    assert np.array_equal(a, b)


def test_full_size_at_solution(ctx):
    """Clustered 128^3 (2.1 M sites) at its solved weights, 128^3 elements on
    a 128^3 mesh: tau = 0 gives density 1 exactly (CIC from cell centres);
    at tau = 0.5 the mass is conserved and the deposit equals the oracle's
    cloud-in-cell assignment of q + tau disp, with disp from
    mak_legendre_mesh (itself matched to the oracle's brute-force Legendre
    transform on sampled nodes here)."""
    import torch
    import paper_2110_08868_amd as mak
    n = 128
    x = workloads.clustered(n, rms=3.0, smooth=1.0, frac=0.2, n_clumps=2000, a=0.5, seed=3)
    sctx = mak.Context(0, "mixed", cg_rtol=1e-3)
    xd = torch.from_numpy(x).cuda()
    psi_d, _, _, info = sctx.solve(xd, 1.0, 1e-6)
    sctx.close()
    r0 = ctx.za_deposit(xd, psi_d, 1.0, 0.0, n, n, "cic", 0.5).cpu().numpy()
    assert np.all(r0 == 1.0)
    tau = 0.5
    r = ctx.za_deposit(xd, psi_d, 1.0, tau, n, n, "cic", 0.5).cpu().numpy()
    assert r.sum() / n ** 3 == pytest.approx(1.0, rel=1e-13)
    phi, idx, disp = ctx.legendre_mesh(xd, psi_d, 1.0, n, 0.5)
    disp = disp.cpu().numpy()
    q = workloads.mesh_points(n, 1.0, 0.5)
    # the located displacements on sampled nodes against the oracle's brute force
    sel = np.random.default_rng(5).choice(n ** 3, 6, replace=False)
    rphi, ridx, rdisp = oracle.legendre(x, psi_d.cpu().numpy(), 1.0, q[sel])
    assert np.abs(phi.cpu().numpy()[sel] - rphi).max() <= 1e-13
    same = idx.cpu().numpy()[sel] == ridx
    assert np.abs(disp[sel][same] - rdisp[same]).max(initial=0) <= 1e-13
    y = np.mod(q + tau * disp, 1.0)
    y[y >= 1.0] = 0.0
    ref = oracle.mesh_assign(y, 1.0 / n ** 3, 1.0, n, "cic").ravel()
    err = np.abs(r.ravel() - ref).max()
    print(f"  rho range {r.min():.3f}..{r.max():.1f}, max |drho| {err:.2e}", flush=True)
    assert err <= 4.0 * n ** 3 / units(n) + 1e-10


def test_errors(ctx):
    import torch
    import paper_2110_08868_amd as mak
    x = torch.from_numpy(workloads.zeldovich(4, rms=0.3, smooth=1.0, seed=77))
    for args in ((1.5, 8, 8, "cic"), (-0.1, 8, 8, "ngp"), (0.5, 0, 8, "cic"), (0.5, 8, 0, "cic")):
        with pytest.raises(mak.MakError) as e:
            ctx.za_deposit(x, None, 1.0, *args)
        assert e.value.name == "MAK_EINVAL"
    ctx.za_deposit(x, None, 1.0, 0.5, 8, 8, "cic")


def test_converges_to_the_moved_cells(ctx):
    """The element deposit (NGP) against the exact deposit of the moved cells
    (the oracle's polytopes clipped against the voxels): the mean error falls
    at first order in the Lagrangian spacing."""
    x = workloads.zeldovich(4, rms=0.5, smooth=1.0, seed=81)
    psi = np.random.default_rng(81).uniform(-1, 1, 64) * 0.03 / 16
    ex = oracle.za_deposit_exact(x, psi, 1.0, 0.5, 6)
    errs = []
    for n_lag in (16, 32, 64, 128):
        r = gdep(ctx, x, psi, 1.0, 0.5, n_lag, 6, "ngp")
        errs.append(float(np.abs(r - ex).mean()))
    print(f"  mean |rho - rho_cells| for n_lag 16..128: {errs}", flush=True)
    for k in range(3):
        assert errs[k + 1] < 0.7 * errs[k]
    assert errs[-1] < 0.03
