"""Closed-form Laguerre diagrams used as pins (derived from Eq. laguerrecell).

Layered product configuration: every site of layer a has x-coordinate X_a and
weight psi_a and sits on a common regular ny x nz yz-lattice.  The power
distance splits into an x part and a yz part,
    min_{a,bc} [1/2 (q_x - X_a)^2 - psi_a + 1/2 |q_yz - y_bc|^2]
  = min_a [1/2 (q_x - X_a)^2 - psi_a] + min_bc 1/2 |q_yz - y_bc|^2,
so each cell is (1-D periodic power interval of its layer) x (yz square).
The interval of layer a is [b_{a-1}, b_a] with
    b_a = (X_a + X_{a+1}) / 2 + (psi_a - psi_{a+1}) / (X_{a+1} - X_a)
(cyclic, X_n = X_0 + L, psi_n = psi_0).

Equal widths L/n give the optimal-transport solution for uniform masses:
    b_0 = sum_a d_a (p_a - a L / n) / L,   b_a = b_0 + a L / n,
    psi_{a+1} = psi_a - d_a (b_a - p_a),
with d_a = X_{a+1} - X_a and p_a the midpoints (the cycle condition
sum_a (psi_a - psi_{a+1}) = 0 fixes b_0).
"""
from __future__ import annotations

import numpy as np


def layer_bounds(X, psi_layer, L):
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Xn = np.append(X, X[0] + L)
    pn = np.append(psi_layer, psi_layer[0])
    d = Xn[1:] - Xn[:-1]
    b = 0.5 * (Xn[:-1] + Xn[1:]) + (pn[:-1] - pn[1:]) / d
    # interval of layer a: [b_{a-1}, b_a]; b_{-1} = b_{n-1} - L
    lo = np.roll(b, 1)
    lo[0] -= L
    return lo, b, d


def layered_cells(X, psi_layer, ny, nz, L):
    """Closed-form volumes, seed-local centroid x-offsets, and the dense J for
    the layered configuration (row order (layer, b, c), c fastest)."""
    X = np.asarray(X, dtype=np.float64)
    nl = X.shape[0]
    lo, hi, d = layer_bounds(X, psi_layer, L)
    w = hi - lo
    dy, dz = L / ny, L / nz
    N = nl * ny * nz
    V = np.repeat(w * dy * dz, ny * nz)
    ux = np.repeat(0.5 * (lo + hi) - X, ny * nz)
    J = np.zeros((N, N))

    def idx(a, b, c):
        return ((a % nl) * ny + (b % ny)) * nz + (c % nz)

    for a in range(nl):
        for b in range(ny):
            for c in range(nz):
                i = idx(a, b, c)
                # x faces: area dy*dz, distance d_a (up) / d_{a-1} (down)
                J[i, idx(a + 1, b, c)] -= dy * dz / d[a]
                J[i, idx(a - 1, b, c)] -= dy * dz / d[(a - 1) % nl]
                # in-layer faces: area w_a * dz at distance dy, w_a * dy at dz
                for s in (1, -1):
                    J[i, idx(a, b + s, c)] -= w[a] * dz / dy
                    J[i, idx(a, b, c + s)] -= w[a] * dy / dz
    np.fill_diagonal(J, 0.0)
    J[np.arange(N), np.arange(N)] = -J.sum(axis=1)
    return V, ux, J


def layered_ot_psi(X, L, widths=None):
    """Layer weights psi (psi_0 = 0) and upper layer boundaries b of the
    transport that gives layer a the slab width widths[a] (all L/n when
    omitted; widths sum to L).

    Layer a occupies [b_{a-1}, b_a] with b_a = b_0 + c_a, c_a = sum_{k=1..a}
    widths[k].  The boundary between sites X_a and X_{a+1} (spacing d_a,
    midpoint p_a) sits at b_a when psi_{a+1} - psi_a = -d_a (b_a - p_a); going
    once round the period returns to psi_0, so sum_a d_a (b_a - p_a) = 0,
    which fixes b_0 = sum_a d_a (p_a - c_a) / L."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    w = np.full(n, L / n) if widths is None else np.asarray(widths, dtype=np.float64)
    assert w.shape == (n,) and abs(w.sum() - L) <= 1e-12 * L
    Xn = np.append(X, X[0] + L)
    d = Xn[1:] - Xn[:-1]
    p = 0.5 * (Xn[:-1] + Xn[1:])
    c = np.concatenate([[0.0], np.cumsum(w[1:])])
    b0 = np.sum(d * (p - c)) / L
    b = b0 + c
    psi = np.zeros(n)
    for k in range(n - 1):
        psi[k + 1] = psi[k] - d[k] * (b[k] - p[k])
    return psi, b
