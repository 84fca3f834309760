"""GPU Legendre transform of the weights and point location (mak_legendre,
mak_legendre_mesh) against the brute-force oracle.

phi(q) is unique and compared element by element.  The minimising site is
unique except at ties: where the oracle's minimum beats every other site by
more than the rounding band the indices must be equal; elsewhere the GPU's
site must attain the minimum to within that band (checked with the minimal
image distance of that site)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

# |phi| is at most a few L^2 here; both sides evaluate 1/2 |d|^2 - psi in
# float64 with a different rounding order: a few ulps of L^2.
ATOL = 1e-13


@pytest.fixture(scope="module")
def ctx():
    import paper_2110_08868_amd as mak
    c = mak.Context(0)
    yield c
    c.close()


def value_at(x, psi, L, q, idx):
    """1/2 |q - x_idx|^2 (nearest image) - psi_idx."""
    d = np.asarray(x)[idx] - q
    d -= L * np.round(d / L)
    return 0.5 * np.sum(d * d, axis=1) - np.asarray(psi)[idx]


def compare(x, psi, L, q, phi, idx, disp, min_match=0.99):
    rphi, ridx, rdisp = oracle.legendre(x, psi, L, q)
    scale = max(1.0, L * L)
    dphi = np.abs(phi - rphi)
    assert dphi.max() <= ATOL * scale, f"phi differs by {dphi.max():.3e}"
    assert idx.min() >= 0 and idx.max() < len(x)
    # the GPU's site attains the minimum
    v = value_at(x, psi, L, np.mod(q, L), idx)
    assert np.max(v - rphi) <= ATOL * scale
    same = idx == ridx
    print(f"  Q={len(q)} max|dphi|={dphi.max():.2e} same index {same.mean():.4f}", flush=True)
    assert same.mean() >= min_match
    assert np.abs(disp[same] - rdisp[same]).max(initial=0) <= 1e-13 * L
    # a different index only at a tie: the oracle's own site is as good
    if not same.all():
        vr = value_at(x, psi, L, np.mod(q[~same], L), ridx[~same])
        assert np.max(np.abs(vr - v[~same])) <= 2 * ATOL * scale
    # disp is the image of the GPU's site relative to q
    img = np.asarray(x)[idx] - np.mod(q, L)
    assert np.allclose(np.mod(disp - img + L / 2, L) - L / 2, 0.0, atol=1e-12)


def run(ctx, x, psi, L, q):
    import torch
    phi, idx, disp = ctx.legendre(torch.from_numpy(x), None if psi is None else torch.from_numpy(psi),
                                  L, torch.from_numpy(q))
    return phi.cpu().numpy(), idx.cpu().numpy().astype(np.int64), disp.cpu().numpy()


def run_mesh(ctx, x, psi, L, ng, off):
    import torch
    phi, idx, disp = ctx.legendre_mesh(torch.from_numpy(x), torch.from_numpy(psi), L, ng, off)
    return phi.cpu().numpy(), idx.cpu().numpy().astype(np.int64), disp.cpu().numpy()


@pytest.mark.parametrize("wscale", [0.0, 0.03, 0.3])
def test_random_queries(ctx, wscale):
    """Zel'dovich 8^3, random weights (0.3: many empty cells), queries spread
    over three periods so that wrapping is exercised."""
    n = 8
    x = workloads.zeldovich(n, rms=0.6, smooth=1.0, seed=31)
    rng = np.random.default_rng(31)
    psi = rng.uniform(-1, 1, len(x)) * wscale / n ** 2
    q = rng.uniform(-1.0, 2.0, (3000, 3))
    compare(x, psi, 1.0, q, *run(ctx, x, psi, 1.0, q))


@pytest.mark.parametrize("ng,off", [(10, 0.0), (12, 0.5), (1, 0.25), (7, 0.3)])
def test_mesh(ctx, ng, off):
    """Mesh nodes, ragged brick tails (ng not a multiple of 4) and ng = 1."""
    n = 6
    L = 2.0
    x = workloads.zeldovich(n, L=L, rms=0.5, smooth=1.0, seed=33)
    rng = np.random.default_rng(33)
    psi = rng.uniform(-1, 1, len(x)) * 0.03 * (L / n) ** 2
    q = workloads.mesh_points(ng, L, off)
    compare(x, psi, L, q, *run_mesh(ctx, x, psi, L, ng, off))


def test_mesh_equals_queries(ctx):
    """The mesh form and the query form give the same bits on the same nodes."""
    x = workloads.clustered(12, seed=35)
    rng = np.random.default_rng(35)
    psi = rng.uniform(-1, 1, len(x)) * 0.02 / 144
    ng, off = 20, 0.5
    a = run_mesh(ctx, x, psi, 1.0, ng, off)
    b = run(ctx, x, psi, 1.0, workloads.mesh_points(ng, 1.0, off))
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_clustered_and_single_site(ctx):
    x = workloads.clustered(10, seed=37)
    rng = np.random.default_rng(37)
    psi = rng.uniform(-1, 1, len(x)) * 0.05 / 100
    q = rng.uniform(0, 1, (2000, 3))
    compare(x, psi, 1.0, q, *run(ctx, x, psi, 1.0, q))
    # N = 1: every point belongs to the one cell
    x1 = np.array([[0.3, 0.7, 0.1]])
    phi, idx, disp = run(ctx, x1, np.array([0.25]), 1.0, q)
    assert np.all(idx == 0)
    compare(x1, np.array([0.25]), 1.0, q, phi, idx, disp)


def test_lattice_ties(ctx):
    """Mesh nodes on the corners of the lattice cells: eight sites tie; phi is
    3/8 s^2 everywhere and the index one of the eight."""
    n = 4
    s = 1.0 / n
    x = workloads.lattice(n)
    q = workloads.mesh_points(n, 1.0, 0.0)
    phi, idx, disp = run(ctx, x, np.zeros(len(x)), 1.0, q)
    assert np.allclose(phi, 3.0 / 8.0 * s * s, rtol=1e-14)
    assert np.allclose(np.abs(disp), 0.5 * s, rtol=1e-14)
    compare(x, np.zeros(len(x)), 1.0, q, phi, idx, disp, min_match=0.0)


def test_psi_none_and_empty(ctx):
    import torch
    x = workloads.zeldovich(4, rms=0.3, smooth=1.0, seed=39)
    q = np.random.default_rng(39).uniform(0, 1, (100, 3))
    a = run(ctx, x, None, 1.0, q)
    b = run(ctx, x, np.zeros(len(x)), 1.0, q)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    phi, idx, disp = ctx.legendre(torch.from_numpy(x), None, 1.0, torch.zeros((0, 3), dtype=torch.float64))
    assert phi.numel() == 0


def test_errors(ctx):
    import torch
    import paper_2110_08868_amd as mak
    x = torch.from_numpy(workloads.zeldovich(4, rms=0.3, smooth=1.0, seed=41))
    q = torch.zeros((5, 3), dtype=torch.float64)
    q[3, 1] = float("nan")
    with pytest.raises(mak.MakError) as e:
        ctx.legendre(x, None, 1.0, q)
    assert e.value.name == "MAK_EINVAL"
    with pytest.raises(mak.MakError) as e:
        ctx.legendre_mesh(x, None, 1.0, 0)
    assert e.value.name == "MAK_EINVAL"
    # still usable
    ctx.legendre_mesh(x, None, 1.0, 4)


def test_full_size_at_solution(ctx):
    """Clustered 128^3 input (2.1 M sites) at its solved weights, mesh 128^3
    with node offset 1/2: sampled nodes against the oracle, and at every node
    the properties that hold at any size: Phi = 1/2 |q|^2 - phi is convex
    along the mesh lines and the transport map q + disp is monotone along
    them."""
    import torch
    import paper_2110_08868_amd as mak
    n = 128
    x = workloads.clustered(n, rms=3.0, smooth=1.0, frac=0.2, n_clumps=2000, a=0.5, seed=3)
    sctx = mak.Context(0, "mixed", cg_rtol=1e-3)
    xd = torch.from_numpy(x).cuda()
    psi_d, _, _, info = sctx.solve(xd, 1.0, 1e-6)
    sctx.close()
    print(f"  solve: {info}", flush=True)
    ng, off = n, 0.5
    phi_d, idx_d, disp_d = ctx.legendre_mesh(xd, psi_d, 1.0, ng, off)
    phi = phi_d.cpu().numpy().reshape(ng, ng, ng)
    idx = idx_d.cpu().numpy().astype(np.int64)
    disp = disp_d.cpu().numpy().reshape(ng, ng, ng, 3)
    psi = psi_d.cpu().numpy()
    # sampled nodes against the oracle
    rng = np.random.default_rng(43)
    pick = rng.choice(ng ** 3, 6, replace=False)
    qn = workloads.mesh_points(ng, 1.0, off)
    rphi, ridx, rdisp = oracle.legendre(x, psi, 1.0, qn[pick])
    assert np.abs(phi.ravel()[pick] - rphi).max() <= ATOL
    v = value_at(x, psi, 1.0, qn[pick], idx[pick])
    assert np.max(v - rphi) <= ATOL
    # convexity of Phi and monotone transport along the three mesh directions
    h = 1.0 / ng
    t = (np.arange(ng) + off) * h
    Q = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1)
    Phi = 0.5 * np.sum(Q * Q, axis=-1) - phi
    for a in range(3):
        d2 = np.diff(Phi, n=2, axis=a)
        assert d2.min() >= -1e-12, f"Phi not convex along axis {a}: {d2.min():.3e}"
        T = Q[..., a] + disp[..., a]
        assert np.diff(T, axis=a).min() >= -1e-12
    # every cell has volume 1/N = one mesh cell: the nodes spread over the
    # cells (a cell holding many nodes would be a wrong location)
    cnt = np.bincount(idx, minlength=len(x))
    assert cnt.sum() == ng ** 3
    print(f"  nodes per cell: max {cnt.max()} empty {np.mean(cnt == 0):.3f} "
          f"one {np.mean(cnt == 1):.3f}", flush=True)
    assert np.mean(cnt == 1) >= 0.3 and cnt.max() <= 64
