"""CPU oracle for the semi-discrete Monge-Ampere-Kantorovich hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package; the product library and its Python
binding never do.  It shares no code with the HIP implementation.

Contents
  cells(x, psi, L)       periodic Laguerre cell pass (C++ FP64, liboracle.so):
                         volumes, first and second moments, faces.
  hessian_dense / hessian_coo
                         J = dV/dpsi from the faces (derived from Eq. SDK:
                         the face between cells i and j moves by dpsi_j/|d|).
  kantorovich(...)       K(psi) of Eq. SDK from the cell integrals.
  solve(x, L, tol)       damped Newton on K (Sec. on MAK reconstruction: K is
                         concave and C^2, maximised by Newton with the
                         Kitagawa-Merigot-Thibert step control), dense Newton
                         step for small N, plain CG otherwise.
  legendre(x, psi, L, q) Legendre transform of the weights at query points:
                         phi(q), the index of the Laguerre cell holding q,
                         and the transport displacement (brute force).
  za_deposit(...)        Zel'dovich advection of the cells' mass elements
                         and their deposit on an Eulerian mesh;
                         za_deposit_exact: the moved cells clipped against
                         the voxels (the limit of many elements);
                         mesh_assign: NGP / cloud-in-cell assignment of
                         point masses to the mesh.
  power_spectrum(f, L)   shell-averaged power spectrum of a periodic mesh
                         field (FFT estimator, optional window and contrast).
  exact                  exact-rational mini oracle (Python fractions).
"""
from .cells import cells, cell_faces_dict, load_library
from .legendre import legendre
from .power import power_spectrum
from .deposit import za_deposit, za_deposit_exact, mesh_assign
from .newton import (
    hessian_dense,
    hessian_coo,
    kantorovich,
    centroids_from_moments,
    solve,
    newton_step_dense,
    newton_step_cg,
)

__all__ = [
    "cells",
    "cell_faces_dict",
    "load_library",
    "legendre",
    "power_spectrum",
    "za_deposit",
    "za_deposit_exact",
    "mesh_assign",
    "hessian_dense",
    "hessian_coo",
    "kantorovich",
    "centroids_from_moments",
    "solve",
    "newton_step_dense",
    "newton_step_cg",
]
