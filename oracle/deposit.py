"""Zel'dovich advection of the cells and Eulerian deposition (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2 (last paragraph) and the caption of Fig. 1: each Laguerre cell V_i
is the Lagrangian region whose mass ends at x_i; at growth amplitude tau
(0 initial, 1 final) the Zel'dovich approximation moves the mass element at
q along the straight line to its site, q + tau (x_i(q) - q), and the moved
mass is expressed as a density on an Eulerian mesh.

Reading (the paper gives no discretisation): the mass of the cells is
carried by the n_lag^3 elements at the Lagrangian mesh nodes
((a, b, c) + offset) L / n_lag, each of mass (L / n_lag)^3 (initial density
1), located in its cell by the Legendre transform of the weights and moved
with the image of x_i that attains the minimum.  The Eulerian density at
node (a, b, c) L / ng is the mass assigned to it (nearest grid point, or
cloud in cell: trilinear weights over the 8 nodes around the element) per
cell volume (L / ng)^3.  As n_lag grows this converges to the deposit of
the moved cells (each a copy of V_i shrunk by 1 - tau towards x_i).
"""
from __future__ import annotations

import numpy as np

from .cells import _ptr, load_library
from .legendre import legendre


def za_deposit(x, psi, L: float, tau: float, n_lag: int, ng: int, scheme: str = "cic",
               lag_offset: float = 0.5):
    """Density (ng, ng, ng) of the moved mass elements."""
    t = (np.arange(n_lag) + lag_offset) * (L / n_lag)
    A, B, C = np.meshgrid(t, t, t, indexing="ij")
    q = np.stack([A.ravel(), B.ravel(), C.ravel()], axis=1)
    _, _, disp = legendre(x, psi, L, q)
    y = np.mod(q + tau * disp, L)
    y[y >= L] = 0.0
    return mesh_assign(y, (L / n_lag) ** 3, L, ng, scheme)


def mesh_assign(y, m: float, L: float, ng: int, scheme: str = "cic"):
    """Density (ng, ng, ng) of point masses m at positions y (Q, 3) in
    [0, L)^3 on the periodic mesh of nodes a L / ng: nearest grid point, or
    cloud in cell (the node below the point on each axis takes 1 - f of the
    mass, the node above f, f the point's fractional node coordinate; the
    three axis weights multiply).  Mass per node over the node volume."""
    H = L / ng
    u = np.asarray(y, dtype=np.float64) / H
    rho = np.zeros(ng ** 3)
    if scheme == "ngp":
        i = np.mod(np.floor(u + 0.5).astype(np.int64), ng)
        np.add.at(rho, (i[:, 0] * ng + i[:, 1]) * ng + i[:, 2], m)
    else:
        i0 = np.floor(u)
        f = u - i0
        i0 = i0.astype(np.int64)
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1])
                         * (f[:, 2] if dz else 1 - f[:, 2]))
                    j = np.mod(i0 + np.array([dx, dy, dz]), ng)
                    np.add.at(rho, (j[:, 0] * ng + j[:, 1]) * ng + j[:, 2], m * w)
    return rho.reshape(ng, ng, ng) / H ** 3


def za_deposit_exact(x, psi, L: float, tau: float, ng: int, threads: int = 0, idx=None):
    """Density (ng, ng, ng) of the moved cells themselves: each cell V_i
    shrunk by 1 - tau towards x_i carries its mass |V_i| at density
    1 / (1 - tau)^3; the mass in the voxel [a H - H/2, a H + H/2)^3 of node a
    is the volume of the shrunk polytope inside it (the C++ cell oracle's
    polytope, clipped against the six voxel planes).  tau < 1.  This is the
    limit of za_deposit with scheme 'ngp' as n_lag grows.  idx: deposit only
    these cells (all by default)."""
    assert 0.0 <= tau < 1.0
    x = np.mod(np.ascontiguousarray(x, dtype=np.float64), L)
    x[x >= L] = 0.0
    x = np.ascontiguousarray(x)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    rho = np.zeros(ng ** 3)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
    load_library().oracle_deposit_exact(_ptr(x), _ptr(psi), x.shape[0], float(L), float(tau), int(ng),
                                        None if idx is None else _ptr(idx), 0 if idx is None else len(idx),
                                        _ptr(rho), int(threads))
    return rho.reshape(ng, ng, ng)
