"""Synthetic input generators: determinism and the recipe's stated statistics."""
import math

import numpy as np

import workloads


def test_lattice_layout():
    x = workloads.lattice(4, L=2.0)
    assert x.shape == (64, 3)
    assert np.allclose(x[0], [0.25, 0.25, 0.25])
    assert np.allclose(x[1], [0.25, 0.25, 0.75])  # z fastest
    assert np.all((x >= 0) & (x < 2.0))


def test_zeldovich_deterministic_and_rms():
    a = workloads.zeldovich(16, rms=0.3, smooth=2.0, seed=1)
    b = workloads.zeldovich(16, rms=0.3, smooth=2.0, seed=1)
    c = workloads.zeldovich(16, rms=0.3, smooth=2.0, seed=2)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    q = workloads.lattice(16)
    d = a - q
    d -= np.round(d)  # minimum image, L = 1
    rms = math.sqrt(np.mean(np.sum(d * d, axis=1)))
    assert abs(rms - 0.3 / 16) < 1e-12
    # zero mean displacement (delta(k=0) = 0)
    assert np.all(np.abs(d.mean(axis=0)) < 1e-12)
    assert np.all((a >= 0) & (a < 1))


def test_zeldovich_is_curl_free_gradient_spectrum():
    """Psi = grad inv-Laplacian delta: its divergence is -delta, whose spectrum
    falls as k^-1 exp(-(ks)^2); check the log-slope on large scales."""
    n = 32
    x = workloads.zeldovich(n, rms=0.1, smooth=1.0, seed=4)
    d = x - workloads.lattice(n)
    d -= np.round(d)
    D = 1.0 / n
    k = 2 * np.pi * np.fft.fftfreq(n, d=D)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    div = sum(1j * K * np.fft.fftn(d[:, a].reshape(n, n, n)) for a, K in enumerate((KX, KY, KZ)))
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    p = np.abs(div) ** 2
    s = 1.0 * D
    model = np.where(kk > 0, np.exp(-((kk * s) ** 2)) / np.where(kk > 0, kk, 1), 0)
    sel = (kk > 0) & (kk < 0.5 * np.pi / D)
    ratio = p[sel] / model[sel]
    # white-noise scatter only: binned ratio is flat within noise
    kb = kk[sel]
    edges = np.quantile(kb, [0, 0.33, 0.66, 1.0])
    means = [ratio[(kb >= edges[i]) & (kb <= edges[i + 1])].mean() for i in range(3)]
    assert max(means) / min(means) < 1.3


def test_plummer_redraw_count_and_bounds():
    n = 16
    x = workloads.zeldovich(n, rms=1.0, smooth=1.0, seed=3)
    y = workloads.plummer_redraw(x, frac=0.2, n_clumps=50, a=0.5, n=n, seed=9)
    moved = np.any(x != y, axis=1)
    assert moved.sum() == round(0.2 * n ** 3)
    assert np.all((y >= 0) & (y < 1))
    y2 = workloads.plummer_redraw(x, frac=0.2, n_clumps=50, a=0.5, n=n, seed=9)
    assert np.array_equal(y, y2)


def test_serving_mix():
    reqs = workloads.serving_requests(256, seed=1000)
    ns = np.array([r["n"] for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 128
    assert all(0.5 <= r["rms"] <= 3.0 for r in reqs)
    # log-uniform: median near the geometric mean 64
    assert 45 <= np.median(ns) <= 90
