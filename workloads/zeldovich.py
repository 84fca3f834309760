"""Lattice, Zel'dovich and clustered point sets in a periodic box [0, L)^3.

Recipe (the synthetic stand-in for the paper's N-body particle snapshots):

* lattice sites  q = (k + 1/2) * D,  D = L / n,  k in {0..n-1}^3;
* white noise    w ~ N(0, 1) on the n^3 grid, PCG64(seed);
* spectrum       P(k) = k^-1 * exp(-(k s)^2),  s = smooth * D,  delta(k=0) = 0;
* displacement   Psi_a(k) = -i k_a delta(k) / k^2   (the gradient of the inverse
                 Laplacian of delta), Nyquist plane of each derivative zeroed;
* rescale        so that sqrt(<|Psi|^2>) (3-D vector rms) equals rms * D;
* positions      x = (q + Psi) mod L, with x == L folded back to 0.

`plummer_redraw` moves a fraction of the points into Plummer-profile clumps
(radius r = a / sqrt(u^(-2/3) - 1), rejected above L/4), which gives the very
uneven cell sizes of collapsed haloes.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft


def wrap(x: np.ndarray, L: float) -> np.ndarray:
    """Fold coordinates into [0, L); values that round to L are mapped to 0."""
    y = np.mod(np.asarray(x, dtype=np.float64), L)
    y[y >= L] = 0.0
    return y


def assert_distinct(x: np.ndarray) -> None:
    """Raise if two points coincide exactly (the method needs distinct sites)."""
    u = np.unique(np.ascontiguousarray(x).view([("", x.dtype)] * x.shape[1]))
    if u.shape[0] != x.shape[0]:
        raise ValueError("coincident points in generated input")


def lattice(n: int, L: float = 1.0, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """n^3 lattice sites at (k + 1/2) L/n, translated by `offset`, wrapped; row
    order is x-major (index = (ix * n + iy) * n + iz)."""
    D = L / n
    k = (np.arange(n, dtype=np.float64) + 0.5) * D
    gx, gy, gz = np.meshgrid(k, k, k, indexing="ij")
    q = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    q = q + np.asarray(offset, dtype=np.float64)[None, :]
    return wrap(q, L)


def layered(xs, ny: int, nz: int, L: float = 1.0) -> np.ndarray:
    """Product configuration: every value in `xs` is an x-layer carrying the
    ny x nz yz-lattice ((b + 1/2) L/ny, (c + 1/2) L/nz).  Row order is
    (layer, b, c) with c fastest."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = (np.arange(ny) + 0.5) * (L / ny)
    zs = (np.arange(nz) + 0.5) * (L / nz)
    A, B, C = np.meshgrid(xs, ys, zs, indexing="ij")
    return np.stack([A.ravel(), B.ravel(), C.ravel()], axis=1).astype(np.float64)


def mesh_points(ng: int, L: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """The ng^3 mesh nodes ((a, b, c) + offset) L/ng, a, b, c in [0, ng), in
    row order (a, b, c) with c fastest."""
    k = (np.arange(ng, dtype=np.float64) + offset) * (L / ng)
    A, B, C = np.meshgrid(k, k, k, indexing="ij")
    return np.stack([A.ravel(), B.ravel(), C.ravel()], axis=1)


def _fft_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _displacement(n: int, L: float, smooth: float, rng: np.random.Generator) -> np.ndarray:
    D = L / n
    white = rng.standard_normal((n, n, n))
    wk = scipy.fft.rfftn(white, workers=_fft_workers())
    del white
    kx = 2.0 * np.pi * np.fft.fftfreq(n, d=D)
    kz = 2.0 * np.pi * np.fft.rfftfreq(n, d=D)
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    kk = np.sqrt(k2)
    s = smooth * D
    with np.errstate(divide="ignore", invalid="ignore"):
        pk = np.where(kk > 0, np.exp(-(kk * s) ** 2) / kk, 0.0)
        delta = wk * np.sqrt(pk)
        inv = np.where(k2 > 0, 1.0 / k2, 0.0)
    out = np.empty((3, n, n, n))
    nyq = n // 2 if n % 2 == 0 else None
    for a, K in enumerate((KX, KY, KZ)):
        comp = -1j * K * delta * inv
        if nyq is not None:
            if a == 0:
                comp[nyq, :, :] = 0.0
            elif a == 1:
                comp[:, nyq, :] = 0.0
            else:
                comp[:, :, nyq] = 0.0
        out[a] = scipy.fft.irfftn(comp, s=(n, n, n), axes=(0, 1, 2), workers=_fft_workers())
        del comp
    return out.reshape(3, -1).T.copy()


def zeldovich(n: int, L: float = 1.0, rms: float = 0.3, smooth: float = 2.0,
              seed: int = 1) -> np.ndarray:
    """Lattice of n^3 sites displaced by a seeded Zel'dovich field; `rms` and
    `smooth` are in units of the lattice spacing D = L/n."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = lattice(n, L)
    psi = _displacement(n, L, smooth, rng)
    cur = math.sqrt(float(np.mean(np.sum(psi * psi, axis=1))))
    if cur > 0:
        psi *= (rms * L / n) / cur
    x = wrap(q + psi, L)
    assert_distinct(x)
    return x


def plummer_redraw(x: np.ndarray, frac: float = 0.2, n_clumps: int = 2000,
                   a: float = 0.5, L: float = 1.0, n: int | None = None,
                   seed: int = 3) -> np.ndarray:
    """Move round(frac * N) points (chosen without replacement) into Plummer
    clumps with uniform centres; `a` is the scale radius in lattice spacings
    (n^3 = N unless `n` is given)."""
    x = np.array(x, dtype=np.float64, copy=True)
    N = x.shape[0]
    if n is None:
        n = round(N ** (1.0 / 3.0))
    D = L / n
    rng = np.random.Generator(np.random.PCG64(seed))
    m = int(round(frac * N))
    idx = rng.choice(N, size=m, replace=False)
    centres = rng.uniform(0.0, L, size=(n_clumps, 3))
    which = rng.integers(0, n_clumps, size=m)
    r = np.empty(m)
    filled = 0
    rmax = L / 4.0
    while filled < m:
        u = rng.uniform(0.0, 1.0, size=2 * (m - filled) + 16)
        u = u[u > 0]
        cand = (a * D) / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        cand = cand[np.isfinite(cand) & (cand <= rmax)]
        take = min(cand.size, m - filled)
        r[filled:filled + take] = cand[:take]
        filled += take
    v = rng.standard_normal((m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x[idx] = centres[which] + r[:, None] * v
    x = wrap(x, L)
    assert_distinct(x)
    return x


def clustered(n: int, L: float = 1.0, rms: float = 3.0, smooth: float = 1.0,
              frac: float = 0.2, n_clumps: int = 2000, a: float = 0.5,
              seed: int = 3) -> np.ndarray:
    """Strongly clustered set: Zel'dovich lattice plus Plummer clumps."""
    x = zeldovich(n, L, rms=rms, smooth=smooth, seed=seed)
    return plummer_redraw(x, frac=frac, n_clumps=n_clumps, a=a, L=L, n=n,
                          seed=seed + 7919)


def serving_requests(count: int = 256, seed: int = 1000, n_lo: int = 32,
                     n_hi: int = 128) -> list[dict]:
    """Request mix for the serving workload: lattice side n drawn
    log-uniformly in [n_lo, n_hi] (N = n^3), per-request seed, rms displacement
    uniform in [0.5, 3] lattice spacings, smoothing 1 spacing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        rms = float(rng.uniform(0.5, 3.0))
        out.append({"n": n, "rms": rms, "smooth": 1.0, "seed": seed + r})
    return out
