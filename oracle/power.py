"""Power spectrum of a periodic mesh field (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. BAO reconstruction compares power spectra P(k) of density fields (the
ratios d(k) = P_wig / <P_nw> - 1 and the mode counts N_modes(k) of each
k-bin).  The estimator is the textbook one for a field f sampled on the
periodic ng^3 mesh of side L (spacing H = L / ng):

    delta(k) = H^3 sum_x f(x) exp(-i k . x),   k = 2 pi n / L,
    n the integer frequencies in (-ng/2, ng/2]^3,
    P(k) = |delta(k)|^2 / L^3,

averaged over the modes of each spherical shell: shell j >= 1 holds the
modes with j - 1/2 <= |n| < j + 1/2 (k = 0 belongs to shell 0 and is left
out).  Each shell reports its mode count, the mean |k| and the mean P.

Options: `contrast` treats f as a density and uses f / mean(f) - 1; `window`
p = 1, 2, 3 divides P by W(n)^2 with W(n) = prod_a sinc(pi n_a / ng)^p, the
Fourier window of nearest-grid-point, cloud-in-cell and triangular-shaped-
cloud assignment (sinc x = sin x / x).
"""
from __future__ import annotations

import numpy as np


def power_spectrum(field, L: float, nbins: int | None = None, window: int = 0,
                   contrast: bool = False):
    """(k_mean, power, modes) per shell j = 1..nbins (default ng // 2)."""
    f = np.asarray(field, dtype=np.float64)
    ng = f.shape[0]
    assert f.shape == (ng, ng, ng)
    if nbins is None:
        nbins = ng // 2
    if contrast:
        f = f / f.mean() - 1.0
    H = L / ng
    dk = np.fft.fftn(f) * H ** 3
    P = (dk.real ** 2 + dk.imag ** 2) / L ** 3
    n1 = np.fft.fftfreq(ng, d=1.0 / ng)            # 0, 1, ..., -1 (integers as floats)
    if ng % 2 == 0:
        n1[ng // 2] = ng // 2                      # Nyquist counted as +ng/2
    nx, ny, nz = np.meshgrid(n1, n1, n1, indexing="ij")
    n2 = nx * nx + ny * ny + nz * nz
    if window:
        def sinc(n):
            x = np.pi * n / ng
            out = np.ones_like(x)
            nzm = x != 0
            out[nzm] = np.sin(x[nzm]) / x[nzm]
            return out
        W = (sinc(nx) * sinc(ny) * sinc(nz)) ** window
        P = P / (W * W)
    j = np.floor(np.sqrt(n2) + 0.5).astype(np.int64)
    kmag = 2.0 * np.pi / L * np.sqrt(n2)
    sel = (j >= 1) & (j <= nbins)
    modes = np.bincount(j[sel], minlength=nbins + 1)[1:]
    psum = np.bincount(j[sel], weights=P[sel], minlength=nbins + 1)[1:]
    ksum = np.bincount(j[sel], weights=kmag[sel], minlength=nbins + 1)[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        return ksum / modes, psum / modes, modes
