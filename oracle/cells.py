"""ctypes binding of the C++ oracle cell pass (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def load_library():
    """Load oracle/liboracle.so, building it first if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_cells.restype = P
    lib.oracle_cells.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, P,
                                 ctypes.c_int64, ctypes.c_int]
    lib.oracle_nfaces.restype = ctypes.c_int64
    lib.oracle_nfaces.argtypes = [P]
    lib.oracle_fetch.restype = None
    lib.oracle_fetch.argtypes = [P] * 12
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [P]
    lib.oracle_deposit_exact.restype = None
    lib.oracle_deposit_exact.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int]
    _LIB = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def cells(x, psi, L: float, idx=None, threads: int = 0) -> dict:
    """Laguerre cells of sites `x` (N,3) with weights `psi` (N,) on the torus
    [0, L)^3 (Eq. laguerrecell), computed by clipping against every site and
    periodic image.

    Returns a dict of numpy arrays indexed by position k in `idx` (all cells by
    default):  V (volume), M (first moment, seed-local), S (second moment
    int |q - x_i|^2), R (largest vertex distance), flags (1 empty,
    2 coincident site, 4 image range insufficient), and the faces of cell k at
    face_ptr[k]:face_ptr[k+1]: face_j (other site; == the cell's own index for
    the faces of the [-L/2, L/2]^3 box), face_shift (periodic image),
    face_area, face_dist (|d|), face_b (plane offset, distance b/|d|).
    """
    lib = load_library()
    x = np.ascontiguousarray(x, dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    n = x.shape[0]
    if idx is None:
        idx = np.arange(n, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.shape[0]
    h = lib.oracle_cells(_ptr(x), _ptr(psi), n, float(L), _ptr(idx), m, int(threads))
    try:
        nf = lib.oracle_nfaces(h)
        out = {
            "V": np.empty(m), "M": np.empty((m, 3)), "S": np.empty(m), "R": np.empty(m),
            "flags": np.empty(m, dtype=np.int32),
            "face_ptr": np.empty(m + 1, dtype=np.int64),
            "face_j": np.empty(nf, dtype=np.int32),
            "face_shift": np.empty((nf, 3), dtype=np.int32),
            "face_area": np.empty(nf), "face_dist": np.empty(nf), "face_b": np.empty(nf),
        }
        lib.oracle_fetch(h, _ptr(out["V"]), _ptr(out["M"]), _ptr(out["S"]), _ptr(out["R"]),
                         _ptr(out["flags"]), _ptr(out["face_ptr"]), _ptr(out["face_j"]),
                         _ptr(out["face_shift"]), _ptr(out["face_area"]),
                         _ptr(out["face_dist"]), _ptr(out["face_b"]))
    finally:
        lib.oracle_free(h)
    out["idx"] = idx
    return out


def cell_faces_dict(res: dict, k: int, min_area: float = 0.0, include_box: bool = False) -> dict:
    """Faces of cell k as {(j, sx, sy, sz): (area, dist)} above `min_area`."""
    i = int(res["idx"][k])
    out = {}
    for f in range(res["face_ptr"][k], res["face_ptr"][k + 1]):
        j = int(res["face_j"][f])
        if j == i and not include_box:
            continue
        a = float(res["face_area"][f])
        if a <= min_area:
            continue
        key = (j,) + tuple(int(s) for s in res["face_shift"][f])
        out[key] = (a, float(res["face_dist"][f]))
    return out
