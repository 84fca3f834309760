"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test targets a different kind of mistake (dropped term, wrong sign or
index, transposed operand) in the oracle's cell pass, Hessian or Newton solve.
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import workloads
from oracle import exact
from tests.closed_forms import layered_cells, layered_ot_psi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dyadic_case(seed, n, grid=32, wgrid=1024, wspan=4):
    rng = np.random.default_rng(seed)
    while True:
        xi = rng.integers(0, grid, size=(n, 3))
        if len({tuple(r) for r in xi}) == n:
            break
    pi = rng.integers(-wspan, wspan + 1, size=n)
    xf = xi / grid
    pf = pi / wgrid
    xq = [tuple(Fr(int(v), grid) for v in r) for r in xi]
    pq = [Fr(int(p), wgrid) for p in pi]
    return xf, pf, xq, pq


# ---------------------------------------------------------------- P1 exact
@pytest.mark.parametrize("seed,n", [(5, 8), (11, 12)])
def test_p1_exact_rational(seed, n):
    """FP64 oracle vs exact rational cells on dyadic inputs: volumes, first and
    second moments and face areas to 1e-13 relative, same faces."""
    xf, pf, xq, pq = _dyadic_case(seed, n)
    r = oracle.cells(xf, pf, 1.0)
    for i in range(n):
        e = exact.cell(xq, pq, 1, i)
        assert r["V"][i] == pytest.approx(float(e["V"]), rel=1e-13, abs=1e-16)
        assert np.allclose(r["M"][i], [float(v) for v in e["M"]], rtol=1e-12, atol=1e-16)
        assert r["S"][i] == pytest.approx(float(e["S"]), rel=1e-12, abs=1e-16)
        fo = oracle.cell_faces_dict(r, i, include_box=True)
        fe = {k: exact.area(v) for k, v in e["faces"].items()}
        assert set(fo) == set(fe)
        for k in fe:
            assert fo[k][0] == pytest.approx(fe[k], rel=1e-12, abs=1e-15)


def test_p1_golden_fixture():
    """Stored exact cells (written by tests/golden/make_golden.py from the
    exact oracle) still match the FP64 oracle."""
    g = json.load(open(os.path.join(GOLDEN, "exact_cells_dyadic8.json")))
    x = np.array(g["x"], dtype=np.float64)
    psi = np.array(g["psi"], dtype=np.float64)
    r = oracle.cells(x, psi, g["L"])
    for i, c in enumerate(g["cells"]):
        assert r["V"][i] == pytest.approx(float(Fr(c["V"])), rel=1e-13)
        fo = oracle.cell_faces_dict(r, i)
        fe = {tuple(f["key"]): f["area"] for f in c["faces"]}
        assert set(fo) == set(fe)
        for k in fe:
            assert fo[k][0] == pytest.approx(fe[k], rel=1e-12)


# ---------------------------------------------------------------- P2 lattice
@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("offset", [(0, 0, 0), (0.0123, -0.31, 0.077)])
def test_p2_lattice(n, offset):
    L = 1.0
    D = L / n
    x = workloads.lattice(n, L, offset=offset)
    N = n ** 3
    r = oracle.cells(x, np.zeros(N), L)
    assert np.allclose(r["V"], D ** 3, rtol=1e-13)
    assert np.allclose(r["M"], 0.0, atol=1e-15)
    J = oracle.hessian_dense(r, N)
    if n == 1:
        assert J.shape == (1, 1) and J[0, 0] == 0.0
        return
    nbr = 6 if n >= 3 else 3
    for i in range(N):
        off = np.delete(J[i], i)
        nz = off[np.abs(off) > 1e-12 * D]
        assert len(nz) == nbr
        assert np.allclose(nz, -D * (6 / nbr), rtol=1e-12)
        assert J[i, i] == pytest.approx(6 * D, rel=1e-12)
    for k in range(N):
        faces = oracle.cell_faces_dict(r, k, min_area=1e-12 * D * D, include_box=True)
        assert len(faces) == 6
        assert all(a == pytest.approx(D * D, rel=1e-12) for a, _ in faces.values())


def test_p2_lattice_solve_zero_iterations():
    x = workloads.lattice(4, offset=(0.01, 0.02, 0.03))
    s = oracle.solve(x, 1.0, tol=1e-10)
    assert s["newton_iters"] == 0
    assert np.allclose(s["disp"], 0.0, atol=1e-15)


# ---------------------------------------------------------------- P3 layered
@pytest.mark.parametrize("nl", [2, 3, 5])
def test_p3_layered_cells(nl):
    rng = np.random.default_rng(nl)
    L = 1.0
    X = np.sort(rng.uniform(0, L, nl))
    dmin = np.min(np.diff(np.append(X, X[0] + L)))
    psi_l = rng.uniform(-1, 1, nl) * 0.1 * dmin ** 2
    ny = nz = 4
    x = workloads.layered(X, ny, nz, L)
    psi = np.repeat(psi_l, ny * nz)
    r = oracle.cells(x, psi, L)
    V, ux, J = layered_cells(X, psi_l, ny, nz, L)
    assert np.all(V > 0)
    assert np.allclose(r["V"], V, rtol=1e-12, atol=1e-15)
    u = r["M"] / r["V"][:, None]
    assert np.allclose(u[:, 0], ux, rtol=1e-11, atol=1e-13)
    assert np.allclose(u[:, 1:], 0.0, atol=1e-13)
    Jo = oracle.hessian_dense(r, len(x))
    assert np.allclose(Jo, J, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------- P4 layered OT
def test_p4_layered_ot_solution():
    rng = np.random.default_rng(7)
    L = 1.0
    nl, ny = 6, 4
    X = np.sort(rng.uniform(0, L, nl))
    psi_l, b = layered_ot_psi(X, L)
    x = workloads.layered(X, ny, ny, L)
    N = len(x)
    psi = np.repeat(psi_l, ny * ny)
    r = oracle.cells(x, psi, L)
    assert np.allclose(r["V"], L ** 3 / N, rtol=1e-11)
    # and Newton from psi = 0 lands on the same psi up to a constant
    s = oracle.solve(x, L, tol=1e-10)
    ref = psi - psi.mean()
    assert np.allclose(s["psi"], ref, atol=1e-10)
    cx = np.sort(np.unique(np.round(s["centroids"][:, 0], 9)))
    assert np.allclose(np.diff(cx), L / nl, atol=1e-9)


# ------------------------------------------------ P4b layered OT, given masses
def test_p4b_layered_ot_with_masses():
    """Layers of prescribed, unequal slab widths: the closed-form weights give
    cells of volume width * dy * dz, and Newton with those masses reaches them."""
    rng = np.random.default_rng(11)
    L = 1.0
    nl, ny = 5, 4
    X = np.sort(rng.uniform(0, L, nl))
    w = rng.uniform(0.5, 1.5, nl)
    w *= L / w.sum()
    psi_l, b = layered_ot_psi(X, L, widths=w)
    assert np.allclose(np.diff(b), w[1:])
    x = workloads.layered(X, ny, ny, L)
    psi = np.repeat(psi_l, ny * ny)
    m = np.repeat(w * (L / ny) ** 2, ny * ny)
    r = oracle.cells(x, psi, L)
    assert np.allclose(r["V"], m, rtol=1e-11)
    s = oracle.solve(x, L, tol=1e-11, masses=m)
    assert s["newton_iters"] > 0
    assert np.allclose(s["psi"], psi - psi.mean(), atol=1e-10)
    # uniform widths reduce to the equal-mass solve
    psi_u, _ = layered_ot_psi(X, L, widths=np.full(nl, L / nl))
    assert np.array_equal(psi_u, layered_ot_psi(X, L)[0])


def test_p4c_masses_of_a_weight_vector_recover_it():
    """The dual maximiser is unique up to a constant: solving for the volumes
    V(psi) of a random weight vector returns that vector."""
    x, psi = _random_case(n=4, seed=9, wscale=0.04)
    r = oracle.cells(x, psi, 1.0)
    s = oracle.solve(x, 1.0, tol=1e-12, masses=r["V"])
    assert s["newton_iters"] > 0
    assert np.allclose(s["psi"], psi - psi.mean(), atol=1e-11 / 16)
    with pytest.raises(ValueError):
        oracle.solve(x, 1.0, masses=np.full(len(x), 2.0 / len(x)))
    bad = r["V"].copy()
    bad[0], bad[1] = -bad[0], bad[1] + 2 * bad[0]
    with pytest.raises(ValueError):
        oracle.solve(x, 1.0, masses=bad)


# ---------------------------------------------------------------- P5 invariants
def _random_case(n=6, seed=3, wscale=0.03):
    x = workloads.zeldovich(n, rms=0.6, smooth=1.0, seed=seed)
    rng = np.random.default_rng(seed)
    D = 1.0 / n
    psi = rng.uniform(-1, 1, len(x)) * wscale * D * D
    return x, psi


def test_p5_volume_sum_and_pyramid_identity():
    x, psi = _random_case()
    r = oracle.cells(x, psi, 1.0)
    assert r["V"].sum() == pytest.approx(1.0, rel=1e-12)
    fp = r["face_ptr"]
    for k in range(len(x)):
        sl = slice(fp[k], fp[k + 1])
        h = r["face_b"][sl] / r["face_dist"][sl]
        assert r["V"][k] == pytest.approx(np.sum(r["face_area"][sl] * h) / 3.0, rel=1e-11)


def test_p5_hessian_symmetric_zero_rowsum():
    x, psi = _random_case()
    r = oracle.cells(x, psi, 1.0)
    J = oracle.hessian_dense(r, len(x))
    assert np.abs(J - J.T).max() <= 1e-12 * np.abs(J).max()
    assert np.abs(J.sum(axis=1)).max() <= 1e-13 * np.abs(J).max()
    assert np.all(r["V"] > 0) and np.all(np.diag(J) > 0)


def test_p5_monotone_map():
    """(x_i - x_j')(c_i - c_j') >= 0 across every face (discrete form of the
    convex Brenier potential: no shell crossing)."""
    x, psi = _random_case(seed=5)
    r = oracle.cells(x, psi, 1.0)
    u = r["M"] / r["V"][:, None]
    fp = r["face_ptr"]
    for k in range(len(x)):
        for f in range(fp[k], fp[k + 1]):
            j = r["face_j"][f]
            if j == k:
                continue
            s = r["face_shift"][f]
            xj = x[j] + s
            ci = x[k] + u[k]
            cj = xj + u[j]
            assert np.dot(x[k] - xj, ci - cj) >= -1e-15


def test_p5_psi_shift_translation_permutation_scaling():
    x, psi = _random_case(seed=9)
    N = len(x)
    r = oracle.cells(x, psi, 1.0)
    r2 = oracle.cells(x, psi + 0.37, 1.0)
    assert np.allclose(r2["V"], r["V"], rtol=1e-10)
    t = np.array([0.3, -0.12, 0.71])
    r3 = oracle.cells(workloads.wrap(x + t, 1.0), psi, 1.0)
    assert np.allclose(r3["V"], r["V"], rtol=1e-10)
    perm = np.random.default_rng(1).permutation(N)
    r4 = oracle.cells(x[perm], psi[perm], 1.0)
    assert np.allclose(r4["V"], r["V"][perm], rtol=1e-12)
    lam = 2.5
    r5 = oracle.cells(x * lam, psi * lam ** 2, lam)
    assert np.allclose(r5["V"], r["V"] * lam ** 3, rtol=1e-12)
    assert np.allclose(r5["M"], r["M"] * lam ** 4, rtol=1e-10, atol=1e-15)


# ---------------------------------------------------------------- P6 finite differences
def test_p6_gradient_of_K():
    x, psi = _random_case(seed=13)
    N = len(x)
    m = np.full(N, 1.0 / N)
    r = oracle.cells(x, psi, 1.0)
    g = m - r["V"]
    h = 1e-7
    for i in (0, 17, 101, N - 1):
        e = np.zeros(N)
        e[i] = h
        kp = oracle.kantorovich(oracle.cells(x, psi + e, 1.0), psi + e, m)
        km = oracle.kantorovich(oracle.cells(x, psi - e, 1.0), psi - e, m)
        assert (kp - km) / (2 * h) == pytest.approx(g[i], abs=1e-6 * np.abs(g).max())


def test_p6_hessian_columns():
    x, psi = _random_case(seed=17)
    N = len(x)
    r = oracle.cells(x, psi, 1.0)
    J = oracle.hessian_dense(r, N)
    h = 1e-8
    for j in (3, 50, 150):
        e = np.zeros(N)
        e[j] = h
        col = (oracle.cells(x, psi + e, 1.0)["V"] - oracle.cells(x, psi - e, 1.0)["V"]) / (2 * h)
        assert np.allclose(col, J[:, j], atol=1e-6 * np.abs(J).max())


# ---------------------------------------------------------------- P7 raster
def test_p7_raster_brute_force():
    """Assign a fine grid of sample points to the cell of smallest power
    distance (minimum image); counts times voxel volume approach V."""
    n = 3
    x, psi = _random_case(n=n, seed=21, wscale=0.2)
    r = oracle.cells(x, psi, 1.0)
    M = 96
    h = 1.0 / M
    g = (np.arange(M) + 0.5) * h
    Q = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    best = np.full(Q.shape[0], np.inf)
    owner = np.zeros(Q.shape[0], dtype=np.int64)
    for i in range(len(x)):
        d = Q - x[i]
        d -= np.round(d)
        p = 0.5 * np.sum(d * d, axis=1) - psi[i]
        better = p < best
        best[better] = p[better]
        owner[better] = i
    V = np.bincount(owner, minlength=len(x)) * h ** 3
    # O(h) boundary error: within 1% of the mean cell volume at h = L/96
    assert np.max(np.abs(V - r["V"])) <= 0.01 / len(x)


# ---------------------------------------------------------------- P8 Newton step
def test_p8_dense_vs_cg_newton_step():
    x, psi = _random_case(seed=23)
    N = len(x)
    r = oracle.cells(x, psi, 1.0)
    g = 1.0 / N - r["V"]
    p1 = oracle.newton_step_dense(oracle.hessian_dense(r, N), g)
    p2 = oracle.newton_step_cg(oracle.hessian_coo(r, N), g)
    assert np.allclose(p1 - p1.mean(), p2, atol=1e-8 * np.abs(p1).max())
    J = oracle.hessian_dense(r, N)
    assert np.allclose(J @ p1, g - g.mean(), atol=1e-12)


def test_oracle_solve_small_zeldovich():
    x = workloads.zeldovich(6, rms=0.5, smooth=1.0, seed=31)
    s = oracle.solve(x, 1.0, tol=1e-9)
    assert s["err"] <= 1e-9
    # certificate: recompute the cells at the returned psi
    r = oracle.cells(x, s["psi"], 1.0)
    N = len(x)
    assert np.max(np.abs(r["V"] - 1.0 / N)) * N <= 1e-9
    # the errors fall quadratically at the end
    e = s["errs"]
    assert e[-1] < e[0]


def test_oracle_flags():
    x = workloads.lattice(2)
    x2 = np.vstack([x, x[:1]])
    r = oracle.cells(x2, np.zeros(9), 1.0)
    assert r["flags"][0] & 2
    # a very negative weight empties a cell
    psi = np.zeros(8)
    psi[0] = -10.0
    r = oracle.cells(x, psi, 1.0)
    assert r["flags"][0] & 1 and r["V"][0] == 0.0
    assert r["V"].sum() == pytest.approx(1.0, rel=1e-12)


# ------------------------------------------------ P9 Legendre transform / location
def test_p9_legendre_lattice_closed_form():
    """psi = 0 on the lattice ((k + 1/2) s): phi is half the squared distance to
    the nearest lattice node, per axis, and i(q) is that node."""
    n, L = 4, 1.0
    s = L / n
    x = workloads.lattice(n, L)
    rng = np.random.default_rng(21)
    q = rng.uniform(-0.5, 1.5, (200, 3))
    phi, idx, disp = oracle.legendre(x, np.zeros(len(x)), L, q)
    u = q / s - 0.5
    k = np.round(u)
    f = (u - k) * s
    assert np.allclose(phi, 0.5 * np.sum(f * f, axis=1), rtol=1e-12, atol=1e-15)
    kk = np.mod(k, n).astype(np.int64)
    assert np.array_equal(idx, (kk[:, 0] * n + kk[:, 1]) * n + kk[:, 2])
    assert np.allclose(disp, -f, atol=1e-14)


def test_p9_legendre_layered_closed_form():
    """Layers with the closed-form transport weights: q lies in the slab of the
    layer a with b_{a-1} < q_x - kL < b_a, and phi follows from that layer's
    image and the nearest yz-lattice line."""
    rng = np.random.default_rng(23)
    L, nl, ny = 1.0, 5, 3
    X = np.sort(rng.uniform(0, L, nl))
    w = rng.uniform(0.5, 1.5, nl)
    w *= L / w.sum()
    psi_l, b = layered_ot_psi(X, L, widths=w)
    x = workloads.layered(X, ny, ny, L)
    psi = np.repeat(psi_l, ny * ny)
    q = rng.uniform(0, L, (300, 3))
    phi, idx, disp = oracle.legendre(x, psi, L, q)
    lo = np.concatenate([[b[-1] - L], b[:-1]])
    s = L / ny
    for t in range(len(q)):
        hits = [(a, k) for a in range(nl) for k in (-1, 0, 1)
                if lo[a] < q[t, 0] - k * L < b[a]]
        assert len(hits) == 1
        a, k = hits[0]
        dx = X[a] + k * L - q[t, 0]
        uy, uz = q[t, 1] / s - 0.5, q[t, 2] / s - 0.5
        fy, fz = (uy - np.round(uy)) * s, (uz - np.round(uz)) * s
        ref = 0.5 * (dx * dx + fy * fy + fz * fz) - psi_l[a]
        assert phi[t] == pytest.approx(ref, rel=1e-12, abs=1e-15)
        iy, iz = int(np.round(uy)) % ny, int(np.round(uz)) % ny
        assert idx[t] == (a * ny + iy) * ny + iz
        assert np.allclose(disp[t], [dx, -fy, -fz], atol=1e-14)


def test_p9_legendre_pure_python_brute_force():
    rng = np.random.default_rng(25)
    L = 2.0
    x = rng.uniform(0, L, (7, 3))
    psi = rng.uniform(-0.2, 0.2, 7)
    q = rng.uniform(0, L, (6, 3))
    phi, idx, disp = oracle.legendre(x, psi, L, q)
    for t in range(len(q)):
        best = None
        for i in range(len(x)):
            for kx in (-1, 0, 1):
                for ky in (-1, 0, 1):
                    for kz in (-1, 0, 1):
                        d = [x[i][0] + kx * L - q[t][0], x[i][1] + ky * L - q[t][1],
                             x[i][2] + kz * L - q[t][2]]
                        v = 0.5 * (d[0] ** 2 + d[1] ** 2 + d[2] ** 2) - psi[i]
                        if best is None or v < best[0]:
                            best = (v, i, d)
        assert phi[t] == pytest.approx(best[0], rel=1e-13, abs=1e-15)
        assert idx[t] == best[1]
        assert np.allclose(disp[t], best[2], atol=1e-14)


def test_p9_legendre_raster_matches_cells():
    """Mesh nodes located in cell i: their number times the node volume
    approaches V_i and their mean position the centroid (the C++ cell oracle)."""
    x, psi = _random_case(n=4, seed=27, wscale=0.03)
    L, ng = 1.0, 40
    q = workloads.mesh_points(ng, L, 0.5)
    phi, idx, disp = oracle.legendre(x, psi, L, q)
    r = oracle.cells(x, psi, L)
    cnt = np.bincount(idx, minlength=len(x)) * (L / ng) ** 3
    assert np.sum(np.abs(cnt - r["V"])) <= 0.03 * L ** 3
    assert np.max(np.abs(cnt - r["V"]) / r["V"]) <= 0.2
    # mean displacement x_i - q over the nodes of cell i = minus the centroid offset
    mu = np.stack([np.bincount(idx, weights=disp[:, a], minlength=len(x)) for a in range(3)], 1)
    mu /= np.bincount(idx, minlength=len(x))[:, None]
    ubar = r["M"] / r["V"][:, None]
    big = r["V"] > 0.5 / len(x)
    assert np.max(np.abs(mu[big] + ubar[big])) <= 0.3 / 4


def test_p9_legendre_potential_convex():
    """Phi(q) = 1/2 |q|^2 - phi(q) (Eq. potpot) is a maximum of affine functions
    of q, hence convex along any line, across the box boundary too."""
    x, psi = _random_case(n=3, seed=29, wscale=0.05)
    L = 1.0
    rng = np.random.default_rng(29)
    for _ in range(4):
        q0 = rng.uniform(-0.5, 1.5, 3)
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        t = np.linspace(0, 1.5, 601)
        q = q0[None, :] + t[:, None] * e[None, :]
        phi, _, disp = oracle.legendre(x, psi, L, q)
        Phi = 0.5 * np.sum(q * q, axis=1) - phi
        d2 = Phi[:-2] - 2 * Phi[1:-1] + Phi[2:]
        assert d2.min() >= -1e-12
        # the slope of Phi along e is e . T(q), T(q) = q + disp the image of the
        # minimising site: monotone along the line (no shell crossing)
        slope = (q + disp) @ e
        assert np.diff(slope).min() >= -1e-12
        assert np.diff(slope).max() > 0


# ------------------------------------------------ P10 power spectrum estimator
def _shell_modes(ng, j):
    """Modes n in (-ng/2, ng/2]^3 with j - 1/2 <= |n| < j + 1/2, by enumeration."""
    lo = -((ng - 1) // 2)
    hi = ng // 2
    c = 0
    for a in range(lo, hi + 1):
        for b in range(lo, hi + 1):
            for d in range(lo, hi + 1):
                r2 = a * a + b * b + d * d
                if (j - 0.5) ** 2 <= r2 < (j + 0.5) ** 2:
                    c += 1
    return c


@pytest.mark.parametrize("ng,n0,window", [(16, (1, 2, 0), 0), (12, (3, -1, 2), 2), (9, (2, 2, 1), 1),
                                          (16, (0, 0, 8), 0), (10, (1, 0, 0), 3)])
def test_p10_plane_wave(ng, n0, window):
    """f = A cos(2 pi n0 . x / L + phase): all power in the modes +-n0 (one
    mode when n0 is the Nyquist frequency), A^2 L^3 / 4 each (A^2 L^3 there),
    divided by the window W(n0)^2; the shells hold the enumerated mode counts."""
    L, A, ph = 2.0, 0.7, 0.3
    t = np.arange(ng) * (L / ng)
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    n0 = np.array(n0)
    nyq = ng % 2 == 0 and np.all(np.isin(np.abs(n0), [0, ng // 2]))
    f = A * np.cos(2 * np.pi * (n0[0] * X + n0[1] * Y + n0[2] * Z) / L + (0.0 if nyq else ph))
    k, P, m = oracle.power_spectrum(f, L, nbins=ng, window=window)
    j0 = int(np.floor(np.linalg.norm(n0) + 0.5))
    for j in (1, 2, j0):
        assert m[j - 1] == _shell_modes(ng, j)
    W = 1.0
    for a in n0:
        x = np.pi * a / ng
        W *= (np.sin(x) / x if a else 1.0) ** window
    tot = (A * A * L ** 3 if nyq else 2 * A * A * L ** 3 / 4) / W ** 2
    assert P[j0 - 1] * m[j0 - 1] == pytest.approx(tot, rel=1e-12)
    others = np.delete(P * m, j0 - 1)
    assert np.all(np.abs(others[np.isfinite(others)]) <= 1e-20 * tot * ng ** 3)


def test_p10_parseval_and_contrast():
    """Sum over all shells of modes x P = H^3 sum f^2 - (H^3 sum f)^2 / L^3;
    contrast divides the k != 0 power by mean(f)^2."""
    rng = np.random.default_rng(51)
    ng, L = 12, 3.0
    f = 2.0 + rng.normal(size=(ng, ng, ng))
    H = L / ng
    k, P, m = oracle.power_spectrum(f, L, nbins=int(np.ceil(np.sqrt(3) * ng / 2)) + 1)
    ok = m > 0
    lhs = np.sum(P[ok] * m[ok])
    rhs = H ** 3 * np.sum(f * f) - (H ** 3 * f.sum()) ** 2 / L ** 3
    assert lhs == pytest.approx(rhs, rel=1e-12)
    kc, Pc, mc = oracle.power_spectrum(f, L, contrast=True)
    kk, Pk, mk = oracle.power_spectrum(f, L)
    assert np.allclose(Pc, Pk / f.mean() ** 2, rtol=1e-12)
    # white noise: E P = sigma^2 H^3 (sigma = 1 here)
    assert np.mean(Pk[1:]) == pytest.approx(H ** 3, rel=0.1)


def test_p10_brute_force_dft():
    """ng = 4: explicit triple-sum DFT per mode, binned by enumeration."""
    rng = np.random.default_rng(53)
    ng, L = 4, 1.5
    f = rng.normal(size=(ng, ng, ng))
    H = L / ng
    acc = {}
    for a in range(-1, 3):
        for b in range(-1, 3):
            for c in range(-1, 3):
                s = 0j
                for x in range(ng):
                    for y in range(ng):
                        for z in range(ng):
                            s += f[x, y, z] * np.exp(-2j * np.pi * (a * x + b * y + c * z) / ng)
                p = abs(s * H ** 3) ** 2 / L ** 3
                r = np.sqrt(a * a + b * b + c * c)
                j = int(np.floor(r + 0.5))
                if j >= 1:
                    e = acc.setdefault(j, [0, 0.0, 0.0])
                    e[0] += 1
                    e[1] += p
                    e[2] += 2 * np.pi / L * r
    k, P, m = oracle.power_spectrum(f, L, nbins=3)
    for j in (1, 2, 3):
        assert m[j - 1] == acc[j][0]
        assert P[j - 1] == pytest.approx(acc[j][1] / acc[j][0], rel=1e-12)
        assert k[j - 1] == pytest.approx(acc[j][2] / acc[j][0], rel=1e-13)


# ------------------------------------------------ P11 Zel'dovich deposit
def test_p11_deposit_tau0_uniform_and_mass():
    """tau = 0 leaves the elements in place: a Lagrangian mesh on the
    Eulerian nodes (NGP), or centred between them (CIC), gives density 1;
    at any tau the deposited mass is L^3."""
    x, psi = _random_case(n=3, seed=63, wscale=0.03)
    L = 1.0
    r = oracle.za_deposit(x, psi, L, 0.0, 6, 6, scheme="ngp", lag_offset=0.0)
    assert np.allclose(r, 1.0, rtol=1e-14)
    r = oracle.za_deposit(x, psi, L, 0.0, 6, 6, scheme="cic", lag_offset=0.5)
    assert np.allclose(r, 1.0, rtol=1e-14)
    for tau, sch in ((0.3, "cic"), (0.8, "ngp"), (1.0, "cic")):
        r = oracle.za_deposit(x, psi, L, tau, 10, 7, scheme=sch)
        assert r.sum() * (L / 7) ** 3 == pytest.approx(L ** 3, rel=1e-13)


def test_p11_deposit_cic_one_element_hand_values():
    """Cloud in cell of one element, worked by hand.  One site at
    (0.55, 0.45, 0.35) in the unit box (its cell is the whole box), one
    Lagrangian element (n_lag = 1, offset 0.3) at q = (0.3, 0.3, 0.3), a 4^3
    mesh (H = 0.25).  At tau = 0.5 the element moves half way to the site's
    nearest image: y = (0.425, 0.375, 0.325), i.e. (1.7, 1.5, 1.3) in node
    units.  Cloud in cell gives the node below the weight 1 - f and the node
    above f: x-axis nodes 1, 2 get 0.3, 0.7; y-axis 0.5, 0.5; z-axis 0.7,
    0.3.  The density at a node is 64 (the element's mass 1 per node volume
    1/64) times the product of its three axis weights.  The weights differ
    per axis and are not symmetric in f <-> 1 - f, so swapping the two
    weights, an off-by-one node or transposed axes all fail here."""
    x = np.array([[0.55, 0.45, 0.35]])
    r = oracle.za_deposit(x, np.zeros(1), 1.0, 0.5, 1, 4, scheme="cic", lag_offset=0.3)
    wx = {1: 0.3, 2: 0.7}
    wy = {1: 0.5, 2: 0.5}
    wz = {1: 0.7, 2: 0.3}
    want = np.zeros((4, 4, 4))
    for a, pa in wx.items():
        for b, pb in wy.items():
            for c, pc in wz.items():
                want[a, b, c] = 64.0 * pa * pb * pc
    assert want[1, 1, 1] == pytest.approx(6.72) and want[2, 2, 2] == pytest.approx(6.72)
    assert want[2, 1, 1] == pytest.approx(15.68) and want[1, 1, 2] == pytest.approx(2.88)
    assert np.allclose(r, want, rtol=1e-12, atol=1e-12)
    # tau = 0: the element stays at (1.2, 1.2, 1.2): weights 0.8 / 0.2 on every axis
    r0 = oracle.za_deposit(x, np.zeros(1), 1.0, 0.0, 1, 4, scheme="cic", lag_offset=0.3)
    assert r0[1, 1, 1] == pytest.approx(64 * 0.512, rel=1e-12)
    assert r0[2, 1, 1] == pytest.approx(64 * 0.128, rel=1e-12)
    assert r0[2, 2, 1] == pytest.approx(64 * 0.032, rel=1e-12)
    assert r0[2, 2, 2] == pytest.approx(64 * 0.008, rel=1e-12)
    assert np.count_nonzero(r0) == 8


def test_p11_deposit_cic_first_moment():
    """Cloud in cell reproduces linear functions: per axis, the mass-weighted
    mean node position of the deposit equals the mean moved element position
    for every element whose two nodes do not wrap (none lies in the last
    node interval [L - H, L)).  The sites sit in the lower part of the box and
    tau is near 1, so every moved element lies within reach of its site and
    the precondition holds.  The moved positions come from the Legendre
    transform of the weights (pinned above, P9); the moment identity itself
    does not use the deposit's weights.  A weight swap moves an element's
    moment from u to 2 i0 + 1 - u and fails."""
    rng = np.random.default_rng(71)
    n_sites = 9
    x = rng.uniform(0.05, 0.55, (n_sites, 3))
    psi = rng.uniform(-1, 1, n_sites) * 1e-3
    L, tau, n_lag, ng = 1.0, 0.9, 12, 4
    H = L / ng
    t = (np.arange(n_lag) + 0.5) * (L / n_lag)
    A, B, C = np.meshgrid(t, t, t, indexing="ij")
    q = np.stack([A.ravel(), B.ravel(), C.ravel()], axis=1)
    _, _, disp = oracle.legendre(x, psi, L, q)
    y = np.mod(q + tau * disp, L)
    assert np.all(y < L - H) and np.all(y >= 0)
    rho = oracle.za_deposit(x, psi, L, tau, n_lag, ng, scheme="cic")
    mass = rho * H ** 3
    assert mass.sum() == pytest.approx(L ** 3, rel=1e-13)
    pos = np.arange(ng) * H
    for ax in range(3):
        node_moment = np.tensordot(mass.sum(axis=tuple(a for a in range(3) if a != ax)), pos, 1)
        assert node_moment == pytest.approx(y[:, ax].sum() * (L / n_lag) ** 3, rel=1e-12)


def _layer_setup():
    rng = np.random.default_rng(61)
    L, nl, ny = 1.0, 3, 2
    X = np.sort(rng.uniform(0, L, nl))
    w = rng.uniform(0.6, 1.4, nl)
    w *= L / w.sum()
    psi_l, b = layered_ot_psi(X, L, widths=w)
    return L, nl, ny, X, psi_l, b


def test_p11_deposit_layered_separable():
    """Slabs with the closed-form transport weights: cells are products of a
    slab in x and lattice squares in y, z, and the Zel'dovich map moves each
    coordinate towards the site's, so the NGP deposit is the product of three
    1-D deposits computed from the slab boundaries; and it approaches the
    exact deposit of the shrunk cells as the Lagrangian mesh refines."""
    L, nl, ny, X, psi_l, b = _layer_setup()
    x = workloads.layered(X, ny, ny, L)
    psi = np.repeat(psi_l, ny * ny)
    ng, tau = 8, 0.4
    H = L / ng
    lo = np.concatenate([[b[-1] - L], b[:-1]])
    s = L / ny

    def fx(n):
        cnt = np.zeros(ng)
        for t in range(n):
            q = (t + 0.5) * L / n
            hit = [(a, k) for a in range(nl) for k in (-1, 0, 1) if lo[a] < q - k * L < b[a]]
            a, k = hit[0]
            y = q + tau * (X[a] + k * L - q)
            cnt[int(np.floor(np.mod(y, L) / H + 0.5)) % ng] += 1
        return cnt

    def fyz(n):
        cnt = np.zeros(ng)
        for t in range(n):
            q = (t + 0.5) * L / n
            k = int(np.floor(q / s))
            y = q + tau * ((k + 0.5) * s - q)
            cnt[int(np.floor(np.mod(y, L) / H + 0.5)) % ng] += 1
        return cnt

    def exact_1d(intervals):
        out = np.zeros(ng)
        for e in range(ng):
            a0, a1 = e * H - H / 2, e * H + H / 2
            for (u0, u1) in intervals:
                for k in (-2, -1, 0, 1, 2):
                    out[e] += max(0.0, min(a1, u1 + k * L) - max(a0, u0 + k * L))
        return out / ((1 - tau) * H)

    ex = exact_1d([(X[a] + (1 - tau) * (lo[a] - X[a]), X[a] + (1 - tau) * (b[a] - X[a]))
                   for a in range(nl)])
    ey = exact_1d([((k + 0.5) * s - (1 - tau) * s / 2, (k + 0.5) * s + (1 - tau) * s / 2)
                   for k in range(ny)])
    exact = ex[:, None, None] * ey[None, :, None] * ey[None, None, :]
    errs = []
    for n in (24, 48):
        r = oracle.za_deposit(x, psi, L, tau, n, ng, scheme="ngp")
        f1, f2 = fx(n), fyz(n)
        ref = f1[:, None, None] * f2[None, :, None] * f2[None, None, :] * (L / n) ** 3 / H ** 3
        assert np.allclose(r, ref, rtol=1e-13, atol=1e-13)
        errs.append(np.abs(r - exact).max())
    assert errs[1] < 0.7 * errs[0] and errs[1] < 0.5


def test_p11_exact_deposit_pins():
    """The exact deposit of the moved cells: density 1 at tau = 0 (the cells
    tile the box), mass L^3 at any tau, the closed form of the layered slabs
    (a product of three 1-D slab averages), and the element deposit (NGP)
    approaching it at first order in the Lagrangian spacing."""
    x, psi = _random_case(n=3, seed=83, wscale=0.03)
    L = 1.0
    assert np.allclose(oracle.za_deposit_exact(x, psi, L, 0.0, 5), 1.0, rtol=1e-12)
    r = oracle.za_deposit_exact(x, psi, L, 0.6, 7)
    assert r.sum() * (L / 7) ** 3 == pytest.approx(L ** 3, rel=1e-12)
    # layered slabs: exact closed form
    L, nl, ny, X, psi_l, b = _layer_setup()
    xl = workloads.layered(X, ny, ny, L)
    ng, tau = 8, 0.4
    H = L / ng
    lo = np.concatenate([[b[-1] - L], b[:-1]])
    s = L / ny

    def slab_avg(intervals):
        out = np.zeros(ng)
        for e in range(ng):
            a0, a1 = e * H - H / 2, e * H + H / 2
            for (u0, u1) in intervals:
                for k in (-2, -1, 0, 1, 2):
                    out[e] += max(0.0, min(a1, u1 + k * L) - max(a0, u0 + k * L))
        return out / ((1 - tau) * H)

    ex = slab_avg([(X[a] + (1 - tau) * (lo[a] - X[a]), X[a] + (1 - tau) * (b[a] - X[a])) for a in range(nl)])
    ey = slab_avg([((k + 0.5) * s - (1 - tau) * s / 2, (k + 0.5) * s + (1 - tau) * s / 2) for k in range(ny)])
    exact = ex[:, None, None] * ey[None, :, None] * ey[None, None, :]
    r = oracle.za_deposit_exact(xl, np.repeat(psi_l, ny * ny), L, tau, ng)
    assert np.allclose(r, exact, rtol=1e-11, atol=1e-12)
    # elements -> cells
    x = workloads.zeldovich(4, rms=0.5, smooth=1.0, seed=81)
    psi = np.random.default_rng(81).uniform(-1, 1, 64) * 0.03 / 16
    ex = oracle.za_deposit_exact(x, psi, 1.0, 0.5, 6)
    e12 = np.abs(oracle.za_deposit(x, psi, 1.0, 0.5, 12, 6, scheme="ngp") - ex).mean()
    e24 = np.abs(oracle.za_deposit(x, psi, 1.0, 0.5, 24, 6, scheme="ngp") - ex).mean()
    assert e24 < 0.65 * e12


def test_p11_exact_deposit_cell_subsets():
    """The exact deposit restricted to cell subsets: the deposits of a
    partition of the cells add up to the full deposit, and each part holds
    exactly its cells' volumes (each cell's mass lands on the mesh whole)."""
    x, psi = _random_case(n=3, seed=87, wscale=0.03)
    L, ng, tau = 1.0, 6, 0.45
    full = oracle.za_deposit_exact(x, psi, L, tau, ng)
    idx = np.random.default_rng(87).permutation(len(x))
    parts = [idx[:7], idx[7:19], idx[19:]]
    got = sum(oracle.za_deposit_exact(x, psi, L, tau, ng, idx=p) for p in parts)
    assert np.allclose(got, full, rtol=1e-12, atol=1e-13)
    vols = oracle.cells(x, psi, L)["V"]
    for p in parts:
        r = oracle.za_deposit_exact(x, psi, L, tau, ng, idx=p)
        assert r.sum() * (L / ng) ** 3 == pytest.approx(vols[p].sum(), rel=1e-12)
