"""GPU parity of mak_laguerre_cells with the CPU oracle (through the C-ABI)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.parity import compare_cells, csr_to_dense, gpu_faces, spacing

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_2110_08868_amd as mak
    c = mak.Context(0)
    yield c
    c.close()


def run(ctx, x, psi, L):
    import torch
    V, C, info = ctx.laguerre_cells(torch.from_numpy(x), torch.from_numpy(psi), L)
    F = gpu_faces(ctx)
    return V.cpu().numpy(), C.cpu().numpy(), F, info


def check(ctx, x, psi, L, hessian=True, **kw):
    print(f"case N={x.shape[0]} L={L} precision={ctx.options['precision']}", flush=True)
    V, C, F, info = run(ctx, x, psi, L)
    res = oracle.cells(x, psi, L)
    rep = compare_cells(x, psi, L, V, C, F, res=res, **kw)
    if hessian and x.shape[0] <= 4096:
        rp, col, val = (t.cpu().numpy() for t in ctx.hessian())
        if x.shape[0] <= 1024:
            Jg = csr_to_dense(rp, col, val, x.shape[0])
            Jo = oracle.hessian_dense(res, x.shape[0])
            assert np.abs(Jg - Jo).max() <= 1e-9 * max(np.abs(Jo).max(), 1e-300)
            # A_ij from cell i and A_ji from cell j are computed apart
            assert np.abs(Jg - Jg.T).max() <= 1e-10 * max(np.abs(Jg).max(), 1e-300)
        else:
            import scipy.sparse as sp
            Jg = sp.csr_matrix((val, col, rp), shape=(x.shape[0],) * 2)
            Jo = oracle.hessian_coo(res, x.shape[0])
            assert abs(Jg - Jo).max() <= 1e-9 * abs(Jo).max()
        # columns sorted, zero row sums
        for i in range(min(x.shape[0], 200)):
            c = col[rp[i]:rp[i + 1]]
            assert np.all(np.diff(c) > 0)
        rs = np.add.reduceat(val, rp[:-1]) if len(val) else np.zeros(0)
        assert np.abs(rs).max() <= 1e-12 * max(np.abs(val).max(), 1e-300)
    print(f"  {rep} nnz={info['nnz']} faces={info['faces']} max_faces={info['max_faces']} "
          f"fp64_rerun={info['fp64_rerun_cells']} overflow={info['overflow_cells']}", flush=True)
    return V, C, F, info, rep


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_lattice(ctx, n):
    x = workloads.lattice(n)
    V, C, F, info, rep = check(ctx, x, np.zeros(n ** 3), 1.0)
    assert np.allclose(V, 1.0 / n ** 3, rtol=1e-13)
    assert rep["straddling_faces"] == 0


def test_lattice_translated(ctx):
    x = workloads.lattice(4, offset=(0.0123, -0.31, 0.077))
    check(ctx, x, np.zeros(64), 1.0)


def test_golden_exact(ctx):
    g = json.load(open(os.path.join(GOLDEN, "exact_cells_dyadic8.json")))
    from fractions import Fraction as Fr
    x = np.array(g["x"])
    psi = np.array(g["psi"])
    V, C, F, info = run(ctx, x, psi, g["L"])
    for i, c in enumerate(g["cells"]):
        assert V[i] == pytest.approx(float(Fr(c["V"])), rel=1e-12)


@pytest.mark.parametrize("seed,wscale", [(1, 0.0), (2, 0.02), (3, 0.05)])
def test_zeldovich_16(ctx, seed, wscale):
    n = 16
    x = workloads.zeldovich(n, rms=0.3, smooth=2.0, seed=seed)
    rng = np.random.default_rng(seed)
    psi = rng.uniform(-1, 1, n ** 3) * wscale / n ** 2
    check(ctx, x, psi, 1.0)


def test_strong_displacement_weights(ctx):
    n = 8
    x = workloads.zeldovich(n, rms=1.5, smooth=1.0, seed=7)
    rng = np.random.default_rng(7)
    psi = rng.uniform(-1, 1, n ** 3) * 0.3 / n ** 2
    check(ctx, x, psi, 1.0)


def test_ragged_uniform_and_box_size(ctx):
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 2.5, size=(1000, 3))
    psi = rng.uniform(-1, 1, 1000) * 0.01
    check(ctx, x, psi, 2.5)


def test_clustered(ctx):
    n = 12
    x = workloads.clustered(n, rms=2.0, smooth=1.0, frac=0.2, n_clumps=10, a=0.5, seed=4)
    check(ctx, x, np.zeros(n ** 3), 1.0)


def test_dense_clump(ctx):
    """A few hundred sites in one Plummer clump inside a lattice: the cells
    around the clump are cut by many sites in turn (plane-table compaction)."""
    n = 8
    x = workloads.zeldovich(n, rms=0.3, smooth=1.0, seed=21)
    x = np.vstack([x, workloads.plummer_redraw(np.zeros((400, 3)), frac=1.0, n_clumps=1, a=0.4,
                                               n=n, seed=21)])
    workloads.assert_distinct(x)
    V, C, F, info, rep = check(ctx, x, np.zeros(len(x)), 1.0)
    assert info["max_faces"] > 20


def test_layered_closed_form(ctx):
    from tests.closed_forms import layered_cells
    rng = np.random.default_rng(3)
    X = np.sort(rng.uniform(0, 1, 5))
    dmin = np.min(np.diff(np.append(X, X[0] + 1)))
    psi_l = rng.uniform(-1, 1, 5) * 0.1 * dmin ** 2
    x = workloads.layered(X, 4, 4)
    psi = np.repeat(psi_l, 16)
    V, C, F, info, rep = check(ctx, x, psi, 1.0)
    Vc, ux, J = layered_cells(X, psi_l, 4, 4, 1.0)
    assert np.allclose(V, Vc, rtol=1e-12)


def test_points_outside_box_are_wrapped(ctx):
    x = workloads.zeldovich(6, rms=0.4, smooth=1.0, seed=8)
    shift = np.random.default_rng(8).integers(-3, 4, size=x.shape).astype(np.float64)
    V1, C1, _, _ = run(ctx, x, np.zeros(216), 1.0)
    V2, C2, _, _ = run(ctx, x + shift, np.zeros(216), 1.0)
    assert np.allclose(V1, V2, rtol=1e-12)


def test_empty_cell(ctx):
    x = workloads.zeldovich(5, rms=0.3, smooth=1.0, seed=9)
    psi = np.zeros(125)
    psi[7] = -0.5
    V, C, F, info, rep = check(ctx, x, psi, 1.0)
    assert V[7] == 0.0 and info["empty_cells"] == 1
    assert V.sum() == pytest.approx(1.0, rel=1e-12)


def test_deterministic(ctx):
    x = workloads.zeldovich(10, rms=0.8, smooth=1.0, seed=12)
    psi = np.random.default_rng(12).uniform(-1, 1, 1000) * 0.003
    V1, C1, F1, _ = run(ctx, x, psi, 1.0)
    V2, C2, F2, _ = run(ctx, x, psi, 1.0)
    assert np.array_equal(V1, V2) and np.array_equal(C1, C2)
    assert np.array_equal(F1["face_area"], F2["face_area"])


def test_errors(ctx):
    import torch

    import paper_2110_08868_amd as mak
    x = workloads.lattice(2)
    dup = np.vstack([x, x[:1]])
    with pytest.raises(mak.MakError) as e:
        ctx.laguerre_cells(torch.from_numpy(dup), torch.zeros(9, dtype=torch.float64), 1.0)
    assert e.value.name == "MAK_EDEGENERATE"
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(mak.MakError) as e:
        ctx.laguerre_cells(torch.from_numpy(bad), torch.zeros(8, dtype=torch.float64), 1.0)
    assert e.value.name == "MAK_EINVAL"
    with pytest.raises(mak.MakError) as e:
        ctx.laguerre_cells(torch.from_numpy(x), torch.zeros(8, dtype=torch.float64), -1.0)
    assert e.value.name == "MAK_EINVAL"
    # the context still works after errors
    check(ctx, x, np.zeros(8), 1.0)


def test_full_size_64_sampled(ctx):
    """64^3 (the mid-size workload) at psi = 0 and at random weights: sampled
    cells against the oracle's one-cell computation, plus global invariants."""
    import torch
    n = 64
    x = workloads.zeldovich(n, rms=1.0, smooth=1.0, seed=2)
    N = n ** 3
    rng = np.random.default_rng(2)
    for psi in (np.zeros(N), rng.uniform(-1, 1, N) * 0.05 / n ** 2):
        V, C, info = ctx.laguerre_cells(torch.from_numpy(x), torch.from_numpy(psi), 1.0)
        V = V.cpu().numpy()
        C = C.cpu().numpy()
        F = gpu_faces(ctx)
        assert V.sum() == pytest.approx(1.0, rel=1e-11)
        idx = rng.choice(N, 64, replace=False)
        res = oracle.cells(x, psi, 1.0, idx=idx)
        rep = compare_cells(x, psi, 1.0, V, C, F, res=res)
        print(f"  64^3 sampled: {rep} nnz={info['nnz']} max_faces={info['max_faces']}", flush=True)
        rp, col, val = (t.cpu().numpy() for t in ctx.hessian())
        rs = np.add.reduceat(val, rp[:-1])
        assert np.abs(rs).max() <= 1e-12 * np.abs(val).max()


# ---------------------------------------------------------------- mixed precision
@pytest.fixture(scope="module")
def mctx():
    import paper_2110_08868_amd as mak
    c = mak.Context(0, "mixed")
    yield c
    c.close()


@pytest.mark.parametrize("case", ["za16", "za16_psi", "clustered12", "lattice4", "uniform1000"])
def test_mixed_precision_parity(mctx, case):
    """Float32 clipping with float64 vertices for the integrals: identical
    adjacency above the area threshold, volumes and centroids to 1e-6 (the
    stated bound; observed far tighter), against the float64 oracle."""
    rng = np.random.default_rng(42)
    if case == "za16":
        x = workloads.zeldovich(16, rms=0.3, smooth=2.0, seed=1)
        psi = np.zeros(len(x))
    elif case == "za16_psi":
        x = workloads.zeldovich(16, rms=1.0, smooth=1.0, seed=2)
        psi = rng.uniform(-1, 1, len(x)) * 0.05 / 256
    elif case == "clustered12":
        x = workloads.clustered(12, rms=2.0, smooth=1.0, frac=0.2, n_clumps=10, a=0.5, seed=4)
        psi = np.zeros(len(x))
    elif case == "lattice4":
        x = workloads.lattice(4, offset=(0.01, 0.02, 0.03))
        psi = np.zeros(len(x))
    else:
        x = rng.uniform(0, 1, size=(1000, 3))
        psi = rng.uniform(-1, 1, 1000) * 0.005
    check(mctx, x, psi, 1.0, vol_rel=1e-6, cen_rel=1e-6, area_rel=1e-6)


def test_mixed_large_cells(mctx):
    """Two hub sites, each ringed by 48 or 110 close sites on a sphere, in a
    displaced lattice: the hubs' cells have 42 and 110 faces, so 80 and 216
    vertices, beyond the float32 stage's 64 (and, for the second, the 128 of
    the next stage): they finish in the float64 fallback kernels; every
    cell to the float64 oracle's bar."""
    n = 6
    h = 1.0 / n
    x = [workloads.zeldovich(n, rms=0.3, smooth=1.0, seed=31)]
    for centre, k in (((1.5 * h, 1.5 * h, 1.5 * h), 48), ((3.5 * h, 3.5 * h, 4.5 * h), 110)):
        i = np.arange(k) + 0.5
        phi = np.arccos(1.0 - 2.0 * i / k)
        th = np.pi * (1.0 + 5.0 ** 0.5) * i
        ring = 0.3 * h * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
        x += [np.asarray(centre)[None, :], np.asarray(centre)[None, :] + ring]
    x = np.mod(np.vstack(x), 1.0)
    workloads.assert_distinct(x)
    V, C, F, info, rep = check(mctx, x, np.zeros(len(x)), 1.0, vol_rel=1e-6, cen_rel=1e-6, area_rel=1e-6)
    assert info["max_faces"] >= 100
    assert info["fp64_rerun_cells"] >= 2
    assert info["overflow_cells"] == 0


# ---------------------------------------------------------------- fallback kernels
@pytest.mark.parametrize("precision,stage", [("fp64", 1), ("mixed", 1), ("mixed", 2)])
def test_fallback_kernels_alone(precision, stage):
    """Every cell through a fallback kernel (the larger polytope / float64
    re-run): the same cells as the oracle, to the float64 bar."""
    import paper_2110_08868_amd as mak
    c = mak.Context(0, precision, first_stage=stage)
    try:
        x = workloads.clustered(12, rms=2.0, smooth=1.0, frac=0.2, n_clumps=10, a=0.5, seed=4)
        psi = np.random.default_rng(3).uniform(-1, 1, len(x)) * 0.02 / 144
        V, C, F, info, rep = check(c, x, psi, 1.0)
        assert info["fp64_rerun_cells"] == 0 or precision == "mixed"
    finally:
        c.close()


def test_pyramid_identity_on_device(ctx):
    """Device-side invariant, independent of the oracle: each cell is the union
    of the pyramids from its site over its faces, V_i = sum_f A_f h_f / 3 with
    h_f = (|d|^2/2 + psi_i - psi_j) / |d| the distance of face f from x_i
    (cells small enough to have no face with an image of their own site)."""
    n = 16
    x = workloads.zeldovich(n, rms=0.6, smooth=1.0, seed=31)
    psi = np.random.default_rng(31).uniform(-1, 1, n ** 3) * 0.05 / n ** 2
    V, C, F, info = run(ctx, x, psi, 1.0)
    fp, fj, fs, fa = F["face_ptr"], F["face_j"], F["face_shift"], F["face_area"]
    i = np.repeat(np.arange(n ** 3), np.diff(fp))
    d = x[fj] + fs * 1.0 - x[i]
    dn = np.linalg.norm(d, axis=1)
    h = (0.5 * dn ** 2 + psi[i] - psi[fj]) / dn
    Vp = np.bincount(i, weights=fa * h / 3.0, minlength=n ** 3)
    assert np.abs(Vp - V).max() <= 1e-10 * V.max()
    assert V.sum() == pytest.approx(1.0, rel=1e-12)


def test_above_2_24_sites():
    """257^3 = 16.97 M sites, above 2^24: the range where each cell keeps 20
    face slots instead of 32, the grid build gives its staging buffers back
    before the pass, and a launch needs a 2-D grid of workgroups.  One float64
    and one mixed pass at psi = 0 and at random weights: 32 sampled cells
    against the oracle (each one clipped against every site and image), the
    volumes summing to L^3 and zero Hessian row sums over every row."""
    import torch
    import paper_2110_08868_amd as mak
    n = 257
    N = n ** 3
    assert N > 2 ** 24
    x = workloads.zeldovich(n, rms=2.0, smooth=1.0, seed=5)
    xd = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(257)
    idx = np.sort(rng.choice(N, 32, replace=False))
    psis = [np.zeros(N), rng.uniform(-1, 1, N) * 0.05 / n ** 2]
    refs = [oracle.cells(x, p, 1.0, idx=idx, threads=16) for p in psis]
    for prec, bar in (("fp64", 1e-10), ("mixed", 1e-6)):
        c = mak.Context(0, prec)
        try:
            for psi, res in zip(psis, refs):
                print(f"case 257^3 {prec} psi max {np.abs(psi).max():.1e}", flush=True)
                V, C, info = c.laguerre_cells(xd, torch.from_numpy(psi).cuda(), 1.0)
                assert abs(V.sum().item() - 1.0) <= 1e-11
                F = gpu_faces(c)
                rep = compare_cells(x, psi, 1.0, V.cpu().numpy(), C.cpu().numpy(), F, res=res,
                                    vol_rel=bar, cen_rel=bar, area_rel=bar)
                del F
                rp, col, val = c.hessian()
                rows = torch.repeat_interleave(torch.arange(N, device=rp.device), rp[1:] - rp[:-1])
                rs = torch.zeros(N, dtype=torch.float64, device=rp.device).index_add_(0, rows, val)
                amax = val.abs().max().item()
                rmax = rs.abs().max().item()
                del rows, rs, rp, col, val
                print(f"  {rep} nnz={info['nnz']} max_faces={info['max_faces']} "
                      f"row sum {rmax / amax:.1e}", flush=True)
                assert rmax <= 1e-12 * amax
        finally:
            c.close()
