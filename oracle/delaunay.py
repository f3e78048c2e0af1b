"""Plain CPU reference for the Delaunay edge flips (Section 2: the step that
makes a triangulation Delaunay again by flipping edges, with exact
predicates).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.
Every predicate is evaluated in exact rational arithmetic (a double converts
to a Fraction exactly), so nothing here depends on rounding. On a periodic
axis every other vertex of an edge's quadrilateral is taken at its image
nearest to the edge's first vertex: its coordinate, or that coordinate plus
or minus the period, rounded to FP64, as the library does (the reading the
predicates are exact on; on an axis that is not periodic the stored
coordinates themselves).

* ``incircle`` / ``orient``: signs of the defining determinants.
* ``lawson``: Lawson's algorithm, one flip at a time from a stack of edges,
  until every interior edge is locally Delaunay. For points in general
  position (no four cocircular on an empty circle) the Delaunay
  triangulation is unique, so any correct flipping order ends at it.
* ``violations``: the definition checked edge by edge (locally Delaunay
  everywhere is Delaunay for a valid triangulation) plus orientation.
* ``brute_force``: the triangles whose circumcircle contains no other point,
  by enumeration (tiny point sets only): the definition itself.
* Refinement (Section 2: quality and size bounds, segments kept, no
  encroached segment) has no unique result, so its reference is the set of
  properties a refined mesh must have, each evaluated exactly:
  ``quality`` (squared circumradius and squared circumradius-to-shortest-edge
  ratio as rationals), ``encroached`` (boundary edges whose diametric circle
  strictly holds the opposite corner), ``area`` and ``segments_covered``.
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


def _image(v, o, period):
    """The image of coordinate v nearest to o on an axis of the given period."""
    if period > 0:
        if v - o > 0.5 * period:
            return v - period
        if v - o < -0.5 * period:
            return v + period
    return v


def _point(mesh, v, base):
    """Coordinates of vertex v at its image nearest to vertex base (FP64)."""
    ax, ay = float(mesh["x"][base]), float(mesh["y"][base])
    return (_image(float(mesh["x"][v]), ax, mesh["px"]), _image(float(mesh["y"][v]), ay, mesh["py"]))


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


def _tri_points(mesh, row):
    p, q, r = (int(v) for v in row)
    return [tuple(map(_F, _point(mesh, v, p))) for v in (p, q, r)]


def quality(mesh, tri):
    """Per triangle (r^2, beta^2) as exact rationals: r the circumradius,
    l_a l_b l_c / (2 |det|) with det the orientation determinant, and beta =
    r / (shortest edge) (Section 2, finding low-quality triangles)."""
    out = []
    for row in np.asarray(tri):
        (ax, ay), (bx, by), (cx, cy) = _tri_points(mesh, row)
        la2 = (cx - bx) ** 2 + (cy - by) ** 2
        lb2 = (cx - ax) ** 2 + (cy - ay) ** 2
        lc2 = (bx - ax) ** 2 + (by - ay) ** 2
        det = (ax - cx) * (by - cy) - (ay - cy) * (bx - cx)
        r2 = la2 * lb2 * lc2 / (4 * det * det)
        out.append((r2, r2 / min(la2, lb2, lc2)))
    return out


def boundary_edges(tri):
    """Edges in exactly one triangle, as (triangle, corner opposite)."""
    return [inc[0] for inc in _edges([tuple(int(v) for v in r) for r in np.asarray(tri)]).values() if len(inc) == 1]


def encroached(mesh, tri) -> list:
    """Boundary edges (t, i) whose diametric circle strictly holds the
    opposite corner: (a - v).(b - v) < 0 (Section 2, encroachment)."""
    tri = np.asarray(tri)
    bad = []
    for t, i in boundary_edges(tri):
        pts = _tri_points(mesh, tri[t])
        v, a, b = pts[i], pts[(i + 1) % 3], pts[(i + 2) % 3]
        if (a[0] - v[0]) * (b[0] - v[0]) + (a[1] - v[1]) * (b[1] - v[1]) < 0:
            bad.append((t, i))
    return bad


def area(mesh, tri) -> Fraction:
    """Exact sum of the triangles' signed areas."""
    total = Fraction(0)
    for row in np.asarray(tri):
        (ax, ay), (bx, by), (cx, cy) = _tri_points(mesh, row)
        total += ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax)) / 2
    return total


def segments_covered(mesh0, mesh1) -> bool:
    """Every boundary edge of mesh1 lies on a boundary edge (segment) of
    mesh0, and each segment's length equals the summed length of the edges on
    it (exact: boundary segments are axis-aligned)."""
    def segs(mesh):
        tri = np.asarray(mesh["tri"])
        out = []
        for t, i in boundary_edges(tri):
            pts = _tri_points(mesh, tri[t])
            out.append((pts[(i + 1) % 3], pts[(i + 2) % 3]))
        return out

    def on(seg, p):
        (ax, ay), (bx, by) = seg
        cross = (bx - ax) * (p[1] - ay) - (by - ay) * (p[0] - ax)
        dot = (p[0] - ax) * (bx - ax) + (p[1] - ay) * (by - ay)
        return cross == 0 and 0 <= dot <= (bx - ax) ** 2 + (by - ay) ** 2

    def length(seg):
        (ax, ay), (bx, by) = seg
        if ax != bx and ay != by:
            raise ValueError("segment not axis-aligned")
        return abs(bx - ax) + abs(by - ay)

    s0 = segs(mesh0)
    covered = [Fraction(0)] * len(s0)
    for e in segs(mesh1):
        hits = [k for k, s in enumerate(s0) if on(s, e[0]) and on(s, e[1])]
        if not hits:
            return False
        covered[hits[0]] += length(e)
    return all(c == length(s) for c, s in zip(covered, s0))


def neighbours(tri):
    """[nt, 3]: the triangle across the edge opposite each corner (-1 on the
    boundary), from sorted vertex pairs; raises on an edge in three or more
    triangles."""
    tri = np.asarray(tri, dtype=np.int64)
    nt = len(tri)
    nv = int(tri.max()) + 1
    b, c = tri[:, [1, 2, 0]], tri[:, [2, 0, 1]]
    flat = (np.minimum(b, c) * nv + np.maximum(b, c)).ravel()
    order = np.argsort(flat, kind="stable")
    same = flat[order][1:] == flat[order][:-1]
    if np.any(same[1:] & same[:-1]):
        raise ValueError("an edge belongs to more than two triangles")
    nbr = -np.ones(3 * nt, dtype=np.int64)
    i = np.nonzero(same)[0]
    nbr[order[i]] = order[i + 1] // 3
    nbr[order[i + 1]] = order[i] // 3
    return nbr.reshape(nt, 3)


def violations_at(mesh, tri, idx) -> list:
    """``violations`` restricted to the triangles idx and their edges (for
    meshes too large to check whole)."""
    tri = np.asarray(tri)
    nbr = neighbours(tri)
    bad = []
    for t in (int(v) for v in idx):
        p, q, r = (int(v) for v in tri[t])
        if orient(_point(mesh, p, p), _point(mesh, q, p), _point(mesh, r, p)) <= 0:
            bad.append(("orientation", t))
        for i in range(3):
            u = int(nbr[t, i])
            if u >= 0 and (_illegal(mesh, tri, t, i, u) or _illegal(mesh, tri, u, int(np.nonzero(nbr[u] == t)[0][0]), t)):
                bad.append(("illegal", t, i))
    return bad
