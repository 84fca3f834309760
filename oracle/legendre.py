"""Legendre transform of the weights and point location (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2, the equation after Eq. laguerrecell: the initial potential at a
Lagrangian point q is the Legendre(-Fenchel) transform of the weights (Eq.
Legendre with the final potential replaced by the discrete weights psi):

    phi(q) = min_i [ 1/2 |q - x_i|^2 - psi_i ],

and the minimiser i(q) is the index of the Laguerre cell (Eq. laguerrecell)
that contains q.  On the flat torus [0, L)^3 the minimum runs over every
periodic image x_i + k L as well; the image term is the same weight psi_i, so
for wrapped q and x_i the minimiser is among the 27 images k in {-1, 0, 1}^3.

The displacement returned with it is x_{i(q)} + k L - q for the minimising
image: the transport map q -> x evaluated at q (Eq. potpot: the map is the
gradient of Phi(q) = 1/2 q^2 - phi(q)), minus q.

Brute force: every query against every site and image.  Ties (equal values)
resolve to the first (site, image) pair in site-major, image order
k = (kx, ky, kz) lexicographic in {-1, 0, 1}^3.
"""
from __future__ import annotations

import numpy as np

_SHIFTS = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)],
                   dtype=np.float64)


def _wrap(v, L):
    v = np.mod(np.asarray(v, dtype=np.float64), L)
    v[v >= L] = 0.0
    return v


def legendre(x, psi, L: float, q, chunk_elems: int = 1 << 22):
    """phi (Q,), idx (Q,) int64, disp (Q, 3) for query points q (Q, 3)."""
    x = _wrap(x, L)
    q = _wrap(q, L)
    psi = np.asarray(psi, dtype=np.float64)
    n, nq = x.shape[0], q.shape[0]
    phi = np.full(nq, np.inf)
    idx = np.full(nq, -1, dtype=np.int64)
    disp = np.zeros((nq, 3))
    sc = max(1, min(n, chunk_elems // 27))                 # sites per chunk
    qc = max(1, chunk_elems // (27 * sc))                  # queries per chunk
    for s in range(0, nq, qc):
        qq = q[s:s + qc]
        r = np.arange(qq.shape[0])
        for j in range(0, n, sc):
            img = x[j:j + sc, None, :] + L * _SHIFTS[None, :, :]   # (m, 27, 3)
            d = img.reshape(1, -1, 3) - qq[:, None, :]               # (c, 27 m, 3)
            v = 0.5 * np.einsum("cij,cij->ci", d, d) - np.repeat(psi[j:j + sc], 27)[None, :]
            k = np.argmin(v, axis=1)
            better = v[r, k] < phi[s:s + qc]                         # first minimum wins
            sel = np.nonzero(better)[0]
            phi[s + sel] = v[sel, k[sel]]
            idx[s + sel] = j + k[sel] // 27
            disp[s + sel] = d[sel, k[sel]]
    return phi, idx, disp
