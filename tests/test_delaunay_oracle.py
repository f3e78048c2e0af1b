"""Pins of the Delaunay reference (oracle/delaunay.py) against the
definition and an independent library: brute-force enumeration of empty
circumcircles equals scipy's Delaunay triangulation (Qhull) on small random
point sets; sequential Lawson flipping of jittered split-square meshes ends
at scipy's triangulation (unique in general position) and passes the
edge-by-edge check, which flags the unflipped input."""
import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I

scipy_spatial = pytest.importorskip("scipy.spatial")


@pytest.fixture(scope="module")
def D():
    import delaunay
    return delaunay


def scipy_tri(x, y):
    d = scipy_spatial.Delaunay(np.stack([x, y], axis=1))
    assert len(d.coplanar) == 0
    t = d.simplices.astype(np.int32)
    # Qhull's orientation is not fixed: make every triangle counter-clockwise
    p = np.stack([x, y], axis=1)
    e1, e2 = p[t[:, 1]] - p[t[:, 0]], p[t[:, 2]] - p[t[:, 0]]
    cr = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    t[cr < 0] = t[cr < 0][:, [0, 2, 1]]
    return t


def test_brute_force_matches_scipy(D):
    rng = np.random.default_rng(0)
    for n in (4, 5, 7, 9, 12):
        for _ in range(10):
            x, y = rng.uniform(size=n), rng.uniform(size=n)
            assert D.canonical(D.brute_force(x, y)) == D.canonical(scipy_tri(x, y))


def test_predicates_on_known_configurations(D):
    assert D.orient((0, 0), (1, 0), (0, 1)) == 1 and D.orient((0, 0), (0, 1), (1, 0)) == -1
    assert D.orient((0, 0), (1, 1), (2, 2)) == 0
    sq = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0)]
    assert D.incircle(*sq, (0.0, 1.0)) == 0          # the fourth corner of the square
    assert D.incircle(*sq, (0.5, 0.5)) == 1 and D.incircle(*sq, (2.0, 2.0)) == -1


@pytest.mark.parametrize("kw", [dict(jitter=0.3, seed=1), dict(jitter=0.3, seed=2, diagonal="random"),
                                dict(jitter=0.2, seed=3, Ny=7, ly=0.5)])
def test_lawson_reaches_scipy_delaunay(D, kw):
    m = I.split_square(9, periodic=(False, False), **kw)
    before = D.violations(m, m["tri"])
    assert any(v[0] == "illegal" for v in before)      # the input is not Delaunay
    tri, flips = D.lawson(m)
    assert flips > 0 and len(tri) == m["nt"]
    assert D.violations(m, tri) == []
    assert D.canonical(tri) == D.canonical(scipy_tri(m["x"], m["y"]))


def test_lawson_on_a_periodic_mesh(D):
    m = I.split_square(10, periodic=(True, True), jitter=0.3, seed=4)
    tri, flips = D.lawson(m)
    assert flips > 0 and len(tri) == m["nt"]
    assert D.violations(m, tri) == []


def test_cocircular_lattice_needs_no_flip(D):
    m = I.split_square(8, periodic=(False, False), diagonal="random", seed=5)
    assert D.violations(m, m["tri"]) == []
    tri, flips = D.lawson(m)
    assert flips == 0 and np.array_equal(tri, m["tri"])


def _mesh(pts, tri, px=0.0, py=0.0):
    pts = np.asarray(pts, dtype=np.float64)
    return {"x": pts[:, 0].copy(), "y": pts[:, 1].copy(), "tri": np.asarray(tri, dtype=np.int32), "px": px, "py": py}


def test_quality_closed_forms(D):
    """Right triangles have their circumcentre at the hypotenuse midpoint:
    legs (1, 1) give r^2 = 1/2 and beta^2 = 1/2; legs (3, 4) give r = 5/2 and
    beta = 5/6. Any triangle has 2 beta = 1 / sin(smallest angle)."""
    from fractions import Fraction
    m = _mesh([[0, 0], [1, 0], [0, 1], [7, 1], [10, 1], [7, 5]], [[0, 1, 2], [3, 4, 5]])
    (r2a, b2a), (r2b, b2b) = D.quality(m, m["tri"])
    assert (r2a, b2a) == (Fraction(1, 2), Fraction(1, 2))
    assert (r2b, b2b) == (Fraction(25, 4), Fraction(25, 36))
    rng = np.random.default_rng(11)
    for _ in range(20):
        p = rng.random((3, 2))
        if np.cross(np.append(p[1] - p[0], 0), np.append(p[2] - p[0], 0))[2] < 0:
            p = p[[0, 2, 1]]
        (_, b2), = D.quality(_mesh(p, [[0, 1, 2]]), [[0, 1, 2]])
        angles = []
        for k in range(3):
            u, v = p[(k + 1) % 3] - p[k], p[(k + 2) % 3] - p[k]
            angles.append(np.arccos(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v)))
        assert abs(2 * np.sqrt(float(b2)) * np.sin(min(angles)) - 1) < 1e-9


def test_encroachment_is_thales(D):
    """A corner on the diametric circle (right angle) does not encroach on the
    opposite boundary edge; an obtuse corner does; an acute one does not."""
    right = _mesh([[0, 0], [2, 0], [1, 1]], [[0, 1, 2]])
    obtuse = _mesh([[0, 0], [2, 0], [1, 0.999]], [[0, 1, 2]])
    acute = _mesh([[0, 0], [2, 0], [1, 1.001]], [[0, 1, 2]])
    assert D.encroached(right, right["tri"]) == []
    # every edge of a lone triangle is a boundary edge; the long one is opposite corner 2
    assert (0, 2) in D.encroached(obtuse, obtuse["tri"])
    assert D.encroached(acute, acute["tri"]) == []


def test_area_and_segments(D):
    from fractions import Fraction
    sq = _mesh([[0, 0], [1, 0], [1, 1], [0, 1]], [[0, 1, 2], [0, 2, 3]])
    assert D.area(sq, sq["tri"]) == 1
    # a vertex inserted on the bottom segment: the boundary is still covered
    split = _mesh([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0]], [[0, 4, 3], [4, 1, 2], [4, 2, 3]])
    assert D.area(split, split["tri"]) == 1
    assert D.segments_covered(sq, split)
    # a vertex above the bottom segment, the triangle below it missing: the
    # boundary edges (0, 4) and (4, 1) lie off the segment
    pts = [[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.125]]
    full = _mesh(pts, [[0, 4, 3], [4, 1, 2], [4, 2, 3], [0, 1, 4]])
    assert D.area(full, full["tri"]) == Fraction(1) and D.segments_covered(sq, full)
    notch = _mesh(pts, [[0, 4, 3], [4, 1, 2], [4, 2, 3]])
    assert D.area(notch, notch["tri"]) == Fraction(15, 16)
    assert not D.segments_covered(sq, notch)
