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
