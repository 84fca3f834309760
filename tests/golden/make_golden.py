"""Write tests/golden/exact_cells_dyadic8.json from the exact-rational oracle.

Input: 8 sites on the dyadic grid (k/32)^3 and weights k/1024 (PCG64 seed 5),
L = 1.  Output per cell: the exact volume (as a fraction string) and the faces
{(j, sx, sy, sz): area} other than the own-image box faces.  Only oracle/ is
called; nothing here comes from the HIP path.
"""
import json
import os
import sys
from fractions import Fraction as Fr

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import exact  # noqa: E402


def main():
    rng = np.random.default_rng(5)
    n = 8
    xi = rng.integers(0, 32, size=(n, 3))
    pi = rng.integers(-4, 5, size=n)
    xq = [tuple(Fr(int(v), 32) for v in r) for r in xi]
    pq = [Fr(int(p), 1024) for p in pi]
    cells = []
    for i in range(n):
        e = exact.cell(xq, pq, 1, i)
        faces = [{"key": list(k), "area": exact.area(v)}
                 for k, v in sorted(e["faces"].items()) if k[0] != i]
        cells.append({"V": str(e["V"]), "M": [str(v) for v in e["M"]], "faces": faces})
    out = {"source": "oracle/exact.py (Eq. laguerrecell on the unit torus)",
           "L": 1.0, "x": (xi / 32).tolist(), "psi": (pi / 1024).tolist(), "cells": cells}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_cells_dyadic8.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
