"""Exact-rational Laguerre cells for tiny inputs (test infrastructure only).

Pins the FP64 oracle (oracle.cpp) without sharing its algorithm or its
rounding: every quantity here is a `fractions.Fraction`.

Definition followed (Eq. laguerrecell on the torus): cell i is the set of u
(seed-local, u = q - x_i) with u . d <= b for every other site j and periodic
image s, d = x_j + s L - x_i, b = |d|^2 / 2 + psi_i - psi_j; the site's own
images give the box [-L/2, L/2]^3.

Algorithm: incremental vertex enumeration ("double description").  The
polytope is a list of vertices, each with the set of planes through it.
Cutting by a plane removes the vertices strictly outside (u.d - b > 0), adds
the plane to the vertices lying exactly on it, and creates a vertex on every
edge joining a strictly-inside vertex to a strictly-outside one (two vertices
span an edge iff they share at least two planes and no third vertex carries
all of the shared planes).  Faces are recovered as the vertex sets of each
plane, sorted by exact angle; volume, first and second moments come from the
tetrahedra (site, v0, v_k, v_k+1) of each face fan, and the exact face area
vector from the shoelace sum.

With inputs on a dyadic grid every number stays rational, so the results are
exact: V_i, int u, int |u|^2 and the face area vectors (the area is the norm
of that vector).
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction as Fr


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def _mul(a, s):
    return (a[0] * s, a[1] * s, a[2] * s)


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


class _Poly:
    def __init__(self, L):
        h = Fr(L) / 2
        self.planes = {}  # key -> (n, b)
        for a in range(3):
            for sg in (1, -1):
                n = [Fr(0)] * 3
                n[a] = Fr(sg) * L
                self.planes[("box", a, sg)] = (tuple(n), Fr(L) * L / 2)
        self.verts = []
        for sx in (1, -1):
            for sy in (1, -1):
                for sz in (1, -1):
                    inc = frozenset({("box", 0, sx), ("box", 1, sy), ("box", 2, sz)})
                    self.verts.append(((sx * h, sy * h, sz * h), inc))

    def r2(self):
        return max(_dot(v, v) for v, _ in self.verts) if self.verts else Fr(0)

    def cut(self, key, n, b) -> bool:
        s = [_dot(v, n) - b for v, _ in self.verts]
        if not any(si > 0 for si in s):
            return False
        self.planes[key] = (n, b)
        new = []
        for (v, inc), si in zip(self.verts, s):
            if si < 0:
                new.append((v, inc))
            elif si == 0:
                new.append((v, inc | {key}))
        for a, (va, ia) in enumerate(self.verts):
            if not s[a] < 0:
                continue
            for c, (vc, ic) in enumerate(self.verts):
                if not s[c] > 0:
                    continue
                common = ia & ic
                if len(common) < 2:
                    continue
                if any(common <= iw for w, (_, iw) in enumerate(self.verts) if w != a and w != c):
                    continue
                t = s[a] / (s[a] - s[c])
                new.append((_add(va, _mul(_sub(vc, va), t)), common | {key}))
        self.verts = new
        return True

    def faces(self):
        """{plane key: vertices ordered counter-clockwise about the outward normal}"""
        out = {}
        for key, (n, _b) in self.planes.items():
            vs = []
            for v, inc in self.verts:
                if key in inc and v not in vs:
                    vs.append(v)
            if len(vs) < 3:
                continue
            c = _mul(functools.reduce(_add, vs), Fr(1, len(vs)))
            ref = _sub(vs[0], c)

            def half(a):
                cr = _dot(_cross(ref, a), n)
                return 0 if (cr > 0 or (cr == 0 and _dot(a, ref) > 0)) else 1

            def cmp(p, q):
                a, b2 = _sub(p, c), _sub(q, c)
                ha, hb = half(a), half(b2)
                if ha != hb:
                    return ha - hb
                cr = _dot(_cross(a, b2), n)
                return -1 if cr > 0 else (1 if cr < 0 else 0)

            vs.sort(key=functools.cmp_to_key(cmp))
            area2 = (Fr(0), Fr(0), Fr(0))
            for k in range(len(vs)):
                area2 = _add(area2, _cross(vs[k], vs[(k + 1) % len(vs)]))
            if area2 == (0, 0, 0):
                continue
            out[key] = (vs, _mul(area2, Fr(1, 2)))
        return out


def cell(x, psi, L, i, K: int = 1) -> dict:
    """Exact cell i of the periodic Laguerre diagram.

    x: list of 3-tuples of Fractions in [0, L); psi: list of Fractions.
    Returns V, M (first moment), S (int |u|^2), faces {(j, sx, sy, sz):
    area vector} (box faces under j = i), all exact, and the float max vertex
    radius R.
    """
    L = Fr(L)
    P = _Poly(L)
    xi = x[i]
    cands = []
    for j in range(len(x)):
        if j == i:
            continue
        for sx in range(-K, K + 1):
            for sy in range(-K, K + 1):
                for sz in range(-K, K + 1):
                    d = _sub(_add(x[j], (sx * L, sy * L, sz * L)), xi)
                    cands.append((_dot(d, d), j, (sx, sy, sz), d))
    cands.sort(key=lambda c: (c[0], c[1], c[2]))
    for d2, j, s, d in cands:
        if d2 == 0:
            raise ValueError("coincident sites")
        b = d2 / 2 + psi[i] - psi[j]
        r2 = P.r2()
        if b >= 0 and b * b >= r2 * d2:  # plane distance >= R: no vertex removed
            continue
        P.cut((j,) + s, d, b)
        if not P.verts:
            break
    faces = P.faces() if P.verts else {}
    V = Fr(0)
    M = (Fr(0), Fr(0), Fr(0))
    S = Fr(0)
    out_faces = {}
    for key, (vs, avec) in faces.items():
        a = vs[0]
        for k in range(1, len(vs) - 1):
            b2, c = vs[k], vs[k + 1]
            vol = _dot(a, _cross(b2, c)) / 6
            V += vol
            M = _add(M, _mul(_add(_add(a, b2), c), vol / 4))
            S += vol / 10 * (_dot(a, a) + _dot(b2, b2) + _dot(c, c) + _dot(a, b2) + _dot(b2, c)
                             + _dot(c, a))
        if key[0] == "box":
            sh = [0, 0, 0]
            sh[key[1]] = key[2]
            fk = (i,) + tuple(sh)
        else:
            fk = key
        out_faces[fk] = avec
    return {"V": V, "M": M, "S": S, "faces": out_faces,
            "R": math.sqrt(float(P.r2())) if P.verts else 0.0}


def area(avec) -> float:
    """Face area from an exact area vector."""
    return math.sqrt(float(_dot(avec, avec)))
