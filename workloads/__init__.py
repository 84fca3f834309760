"""Seeded synthetic point sets for the semi-discrete MAK reconstruction.

This module only *draws inputs*.  It holds none of the method's arithmetic (no
power distances, no cells, no Newton step), so that the CPU oracle and the HIP
path can both consume its output without sharing any computation.

Every generator is deterministic in its arguments (numpy PCG64 streams).

The inputs stand in for the paper's datasets (FastPM / AbacusCosmos particle
snapshots, Fig. 1 and Sec. "BAO reconstruction"), which are not available: a
regular lattice displaced by a Zel'dovich field drawn from a smoothed
power-law spectrum, optionally with part of the points redrawn into Plummer
clumps to mimic collapsed haloes.
"""
from .zeldovich import (
    lattice,
    layered,
    mesh_points,
    zeldovich,
    plummer_redraw,
    clustered,
    wrap,
    assert_distinct,
    serving_requests,
)

__all__ = [
    "lattice",
    "layered",
    "mesh_points",
    "zeldovich",
    "plummer_redraw",
    "clustered",
    "wrap",
    "assert_distinct",
    "serving_requests",
]
