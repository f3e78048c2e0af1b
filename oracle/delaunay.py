"""Plain CPU reference for the Delaunay edge flips (Section 2: the step that
makes a triangulation Delaunay again by flipping edges, with exact
predicates).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.
Every predicate is evaluated in exact rational arithmetic (a double converts
to a Fraction exactly), so nothing here depends on rounding. On a periodic
axis the coordinates of an edge's quadrilateral are unwrapped next to its
first vertex in FP64, as the library does (the reading the predicates are
exact on).

* ``incircle`` / ``orient``: signs of the defining determinants.
* ``lawson``: Lawson's algorithm, one flip at a time from a stack of edges,
  until every interior edge is locally Delaunay. For points in general
  position (no four cocircular on an empty circle) the Delaunay
  triangulation is unique, so any correct flipping order ends at it.
* ``violations``: the definition checked edge by edge (locally Delaunay
  everywhere is Delaunay for a valid triangulation) plus orientation.
* ``brute_force``: the triangles whose circumcircle contains no other point,
  by enumeration (tiny point sets only): the definition itself.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations

import numpy as np


def _F(v):
    return Fraction(float(v))


def orient(a, b, c) -> int:
    """Sign of det [b - a, c - a]: +1 counter-clockwise."""
    (ax, ay), (bx, by), (cx, cy) = [(_F(p[0]), _F(p[1])) for p in (a, b, c)]
    det = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    return (det > 0) - (det < 0)


def incircle(a, b, c, d) -> int:
    """Sign of the in-circle determinant: +1 when d is strictly inside the
    circle through the counter-clockwise a, b, c."""
    (dx, dy) = (_F(d[0]), _F(d[1]))
    rows = []
    for p in (a, b, c):
        u, v = _F(p[0]) - dx, _F(p[1]) - dy
        rows.append((u, v, u * u + v * v))
    (a1, a2, a3), (b1, b2, b3), (c1, c2, c3) = rows
    det = a1 * (b2 * c3 - b3 * c2) - a2 * (b1 * c3 - b3 * c1) + a3 * (b1 * c2 - b2 * c1)
    return (det > 0) - (det < 0)


def _unwrap(d, period):
    if period > 0:
        if d > 0.5 * period:
            d -= period
        elif d < -0.5 * period:
            d += period
    return d


def _point(mesh, v, base):
    """Coordinates of vertex v unwrapped next to vertex base (FP64)."""
    ax, ay = float(mesh["x"][base]), float(mesh["y"][base])
    if v == base:
        return (ax, ay)
    return (ax + _unwrap(float(mesh["x"][v]) - ax, mesh["px"]), ay + _unwrap(float(mesh["y"][v]) - ay, mesh["py"]))


def _edges(tri):
    """Map (min, max) vertex pair -> list of (triangle, corner opposite)."""
    e = {}
    for t, (p, q, r) in enumerate(tri):
        for i, (b, c) in enumerate(((q, r), (r, p), (p, q))):
            e.setdefault((min(b, c), max(b, c)), []).append((t, i))
    return e


def _illegal(mesh, tri, t, i, u) -> bool:
    a, b, c = tri[t][i], tri[t][(i + 1) % 3], tri[t][(i + 2) % 3]
    d = [v for v in tri[u] if v != b and v != c][0]
    return incircle(_point(mesh, a, a), _point(mesh, b, a), _point(mesh, c, a), _point(mesh, d, a)) > 0


def violations(mesh, tri) -> list:
    """Edges (t, i) whose opposite vertex in the neighbour lies strictly inside
    the circumcircle, and triangles that are not counter-clockwise."""
    tri = [tuple(int(v) for v in row) for row in np.asarray(tri)]
    bad = []
    for t, (p, q, r) in enumerate(tri):
        if orient(_point(mesh, p, p), _point(mesh, q, p), _point(mesh, r, p)) <= 0:
            bad.append(("orientation", t))
    for pair, inc in _edges(tri).items():
        if len(inc) > 2:
            bad.append(("nonmanifold", pair))
        if len(inc) != 2:
            continue
        (t, i), (u, j) = inc
        if _illegal(mesh, tri, t, i, u) or _illegal(mesh, tri, u, j, t):
            bad.append(("illegal", t, i))
    return bad


def lawson(mesh):
    """Sequential exact Lawson flipping of mesh["tri"]: (tri [nt, 3], flips)."""
    tri = [list(int(v) for v in row) for row in np.asarray(mesh["tri"])]
    owner = {}
    for pair, inc in _edges(tri).items():
        owner[pair] = [t for t, _ in inc]
    stack = [pair for pair, ts in owner.items() if len(ts) == 2]
    flips = 0
    while stack:
        b, c = stack.pop()
        ts = owner.get((b, c))
        if ts is None or len(ts) != 2:
            continue
        t, u = ts
        i = [k for k in range(3) if tri[t][k] not in (b, c)][0]
        if not _illegal(mesh, tri, t, i, u):
            continue
        a = tri[t][i]
        bb, cc = tri[t][(i + 1) % 3], tri[t][(i + 2) % 3]
        d = [v for v in tri[u] if v != bb and v != cc][0]
        # (a, bb, cc) + (cc, bb, d) -> (a, bb, d) + (d, cc, a)
        tri[t] = [a, bb, d]
        tri[u] = [d, cc, a]
        del owner[(min(bb, cc), max(bb, cc))]
        owner[(min(a, d), max(a, d))] = [t, u]
        for (p, q), old, new in (((bb, d), u, t), ((cc, a), t, u)):
            key = (min(p, q), max(p, q))
            owner[key] = [new if x == old else x for x in owner[key]]
        for p, q in ((a, bb), (bb, d), (d, cc), (cc, a)):
            stack.append((min(p, q), max(p, q)))
        flips += 1
    return np.array(tri, dtype=np.int32), flips


def brute_force(x, y):
    """Delaunay triangles of a small point set in general position: every
    counter-clockwise triple whose circumcircle has no point strictly inside."""
    pts = list(zip(map(float, x), map(float, y)))
    out = []
    for i, j, k in combinations(range(len(pts)), 3):
        o = orient(pts[i], pts[j], pts[k])
        if o == 0:
            continue
        tri = (i, j, k) if o > 0 else (i, k, j)
        if all(incircle(pts[tri[0]], pts[tri[1]], pts[tri[2]], pts[m]) <= 0
               for m in range(len(pts)) if m not in tri):
            out.append(tri)
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def canonical(tri) -> set:
    """Triangles as a set, each rotated to start at its smallest vertex."""
    out = set()
    for row in np.asarray(tri):
        r = [int(v) for v in row]
        k = r.index(min(r))
        out.add(tuple(r[k:] + r[:k]))
    return out
