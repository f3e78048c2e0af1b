"""GPU Delaunay edge flips (rd_delaunay_flip) against the exact CPU
reference (oracle/delaunay.py) and scipy: for points in general position the
Delaunay triangulation is unique, so the flipped triangle set must equal the
reference's exactly; on cocircular lattices (every cell's corners on one
circle) no edge may flip, which needs the exact predicate."""
import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02028_amd import rd as rdmod
    rdmod.lib()
    return rdmod


@pytest.fixture(scope="module")
def D():
    import delaunay
    return delaunay


def scipy_set(D, m):
    """scipy's (Qhull's) Delaunay triangles, made counter-clockwise."""
    from scipy.spatial import Delaunay
    d = Delaunay(np.stack([m["x"], m["y"]], axis=1))
    assert len(d.coplanar) == 0
    return as_ccw_set(D, m, d.simplices)


def ccw(m, tri):
    p = np.stack([m["x"], m["y"]], axis=1)
    e1, e2 = p[tri[:, 1]] - p[tri[:, 0]], p[tri[:, 2]] - p[tri[:, 0]]
    return e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] > 0


def as_ccw_set(D, m, tri):
    tri = np.array(tri, dtype=np.int64)
    bad = ~ccw(m, tri)
    tri[bad] = tri[bad][:, [0, 2, 1]]
    return D.canonical(tri)


def sheared(m, s=0.37):
    m = dict(m)
    m["x"] = m["x"] + s * m["y"]
    return m


CASES = {
    "jitter": lambda: I.split_square(24, periodic=(False, False), jitter=0.3, seed=1),
    "jitter_random_diagonals": lambda: I.split_square(31, periodic=(False, False), jitter=0.3, seed=2,
                                                      diagonal="random"),
    "sheared_lattice": lambda: sheared(I.split_square(20, periodic=(False, False), seed=3)),
    "rectangle": lambda: I.split_square(33, periodic=(False, False), jitter=0.3, seed=4, Ny=11, ly=0.25),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_flips_match_the_exact_reference(rd, D, case):
    m = CASES[case]()
    rd.rd_mesh_validate(m)  # a valid (counter-clockwise) input triangulation
    say(f"delaunay case={case} nt={m['nt']}")
    tri, flips, rounds = rd.rd_delaunay_flip(m)
    ref, ref_flips = D.lawson(m)
    say(f"  gpu: {flips} flips in {rounds} rounds; sequential reference: {ref_flips} flips")
    assert flips > 0 and len(tri) == m["nt"]
    assert D.canonical(tri) == D.canonical(ref)
    assert D.violations(m, tri) == []
    assert D.canonical(tri) == scipy_set(D, m)


def test_periodic_flips(rd, D):
    m = I.split_square(20, periodic=(True, True), jitter=0.3, seed=5)
    rd.rd_mesh_validate(m)
    tri, flips, rounds = rd.rd_delaunay_flip(m)
    ref, _ = D.lawson(m)
    say(f"periodic: {flips} flips in {rounds} rounds")
    assert flips > 0
    assert D.violations(m, tri) == []
    assert D.canonical(tri) == D.canonical(ref)


@pytest.mark.parametrize("N", [17, 257])
def test_cocircular_lattice_is_left_alone(rd, N):
    """Every cell of the split-square lattice is a cyclic quadrilateral (both
    diagonals are Delaunay); the FP64 test cannot decide, the exact one says
    'on the circle', and nothing flips, for either diagonal choice."""
    for kw in (dict(), dict(diagonal="random", seed=6)):
        m = I.split_square(N, periodic=(False, False), **kw)
        tri, flips, rounds = rd.rd_delaunay_flip(m)
        assert flips == 0 and rounds == 0
        assert np.array_equal(tri, m["tri"])
    m = I.split_square(N)  # periodic
    tri, flips, _ = rd.rd_delaunay_flip(m)
    assert flips == 0 and np.array_equal(tri, m["tri"])


def test_large_jittered_mesh_matches_scipy(rd, D):
    import time
    m = I.split_square(1025, periodic=(False, False), jitter=0.25, seed=7, diagonal="random")
    rd.rd_mesh_validate(m)
    t0 = time.perf_counter()
    tri, flips, rounds = rd.rd_delaunay_flip(m)
    el = time.perf_counter() - t0
    say(f"1025^2 points, {m['nt']} triangles: {flips} flips in {rounds} rounds, {el:.2f} s")
    assert flips > 0 and np.all(ccw(m, tri))
    assert D.canonical(tri) == scipy_set(D, m)


def test_flipped_mesh_runs_the_solver(rd):
    m = I.split_square(40, periodic=(False, False), bc=("ghost", "ghost"), jitter=0.3, seed=8)
    tri, flips, _ = rd.rd_delaunay_flip(m)
    assert flips > 0
    m2 = dict(m)
    m2["tri"] = tri
    g = rd.Mesh(m2)
    W = I.ic_uniform(m2, 1.2, 0.3, -0.1, 0.9)
    g.set_state(W)
    g.step_cfl(5, 0.4, rd.B, rd.RK2, rd.FP64)
    assert np.array_equal(g.get_state(), W)
    g.close()


def test_invalid_triangulations_are_refused(rd):
    m = I.split_square(6, periodic=(False, False))
    bad = dict(m)
    bad["tri"] = np.ascontiguousarray(m["tri"][:, [0, 2, 1]])
    with pytest.raises(rd.RDError) as e:
        rd.rd_delaunay_flip(bad)
    assert e.value.status == rd.RD_EINVAL
    bad = dict(m)
    bad["tri"] = np.concatenate([m["tri"], m["tri"][:1]])  # an edge in three triangles
    bad["nt"] = m["nt"] + 1
    with pytest.raises(rd.RDError) as e:
        rd.rd_delaunay_flip(bad)
    assert e.value.status == rd.RD_EINVAL
