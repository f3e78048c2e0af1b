"""Delaunay refinement (Section 2) on the CPU: the library's per-element
bodies (rd_delaunay_kern.h, the code the GPU kernels run) built with g++ and
run one element at a time by a host copy of the refinement loop
(tests/cpp/delaunay_shim.cpp). A refined mesh has no unique form, so the
reference is the set of properties it must have, each checked exactly by the
reference module (oracle/delaunay.py): a valid counter-clockwise
triangulation, Delaunay, every triangle within the size and quality bounds,
no encroached boundary segment, the input's area, its segments covered by
boundary edges and its vertices kept."""
import ctypes as C
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1705_02028_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SQRT2 = 2 ** 0.5


def build_shim():
    """Build tests/cpp/delaunay_shim.cpp and load it."""
    out = os.path.join(tempfile.mkdtemp(prefix="dl_"), "libdl.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                    "-Wno-unknown-pragmas", "-I", os.path.join(ROOT, "paper_1705_02028_amd", "csrc"),
                    os.path.join(HERE, "cpp", "delaunay_shim.cpp"), "-o", out] + oracle.host_sanitize_flags(),
                   check=True)
    L = C.CDLL(out)
    P = C.c_void_p
    L.rdl_refine.argtypes = [P, P, P, C.c_int64, C.c_double, C.c_double, P, P, C.c_int64, C.c_double,
                             C.c_double, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
    L.rdl_refine.restype = C.c_int
    L.rdl_flip.argtypes = [C.c_int64, P, P, C.c_double, C.c_double, C.c_int64, P, P, P]
    L.rdl_flip.restype = C.c_int
    return L


@pytest.fixture(scope="module")
def S():
    return build_shim()


@pytest.fixture(scope="module")
def D():
    import delaunay
    return delaunay


def host_refine(S, m, R, B, max_vertices=20000, max_iterations=1000, morton=False, size_grid=None):
    """rdl_refine (sequential run of the library's bodies): (status, mesh)."""
    nv, nt = int(m["nv"]), int(m["nt"])
    max_t = 2 * max_vertices + nt
    x, y = np.zeros(max_vertices), np.zeros(max_vertices)
    x[:nv], y[:nv] = m["x"], m["y"]
    tri = np.zeros((max_t, 3), dtype=np.int32)
    tri[:nt] = m["tri"]
    cv, ct, ni, nf = C.c_int64(nv), C.c_int64(nt), C.c_int32(), C.c_int64()
    grid = None if size_grid is None else np.ascontiguousarray(size_grid, np.float64)
    gny, gnx = (0, 0) if grid is None else grid.shape
    st = S.rdl_refine(C.byref(cv), x.ctypes.data, y.ctypes.data, max_vertices, float(m["px"]), float(m["py"]),
                      C.byref(ct), tri.ctypes.data, max_t, R, B, None if grid is None else grid.ctypes.data,
                      gnx, gny, max_iterations, int(morton), C.byref(ni), C.byref(nf))
    nv, nt = cv.value, ct.value
    return st, {"x": x[:nv].copy(), "y": y[:nv].copy(), "tri": tri[:nt].copy(), "nv": nv, "nt": nt,
                "px": m["px"], "py": m["py"], "n_iterations": ni.value, "n_flips": nf.value}


def points_in_box(n, w, h, seed):
    """Corners of [0, w] x [0, h] and n seeded uniform points inside, with
    scipy's Delaunay triangulation made counter-clockwise."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    p = np.vstack([[0, 0], [w, 0], [w, h], [0, h], rng.random((n, 2)) * [w, h]])
    t = Delaunay(p).simplices.astype(np.int32)
    e1, e2 = p[t[:, 1]] - p[t[:, 0]], p[t[:, 2]] - p[t[:, 0]]
    neg = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] < 0
    t[neg] = t[neg][:, [0, 2, 1]]
    return {"x": p[:, 0].copy(), "y": p[:, 1].copy(), "tri": t, "nv": len(p), "nt": len(t), "px": 0.0, "py": 0.0}


def wrapped(m):
    """The mesh with coordinates on periodic axes in [0, period)."""
    m = dict(m)
    if m["px"] > 0:
        m["x"] = np.mod(m["x"], m["px"])
    if m["py"] > 0:
        m["y"] = np.mod(m["y"], m["py"])
    return m


CASES = {
    # (input, R, B)
    "square": (lambda: points_in_box(0, 1.0, 1.0, 0), 0.05, SQRT2),
    "random_points": (lambda: points_in_box(40, 1.0, 1.0, 1), 0.1, SQRT2),
    "rectangle_quality_only": (lambda: points_in_box(60, 2.0, 1.0, 2), 0.0, SQRT2),
    "periodic": (lambda: wrapped(I.split_square(8, periodic=(True, True), jitter=0.3, seed=5)), 0.06, SQRT2),
    "periodic_x_walls_y": (lambda: wrapped(I.split_square(7, periodic=(True, False), jitter=0.3, seed=6)),
                           0.08, SQRT2),
}


def check_refined(D, m0, m1, R, B, sample=None, seed=0, morton=False):
    """The properties of a refined mesh, exactly (on a seeded sample of
    `sample` triangles when given); returns a short summary."""
    tri = np.asarray(m1["tri"])
    nv0 = int(m0["nv"])
    if morton:  # the input points are kept, renumbered
        out = set(zip(m1["x"].tolist(), m1["y"].tolist()))
        assert all(p in out for p in zip(m0["x"].tolist(), m0["y"].tolist()))
    else:
        assert np.array_equal(m1["x"][:nv0], m0["x"]) and np.array_equal(m1["y"][:nv0], m0["y"])
    assert tri.min() >= 0 and tri.max() < m1["nv"]
    # every vertex is used
    assert len(np.unique(tri)) == m1["nv"]
    # edges in at most two triangles, Delaunay, counter-clockwise
    # (violations() checks all three; on a sample, only the sampled triangles' edges)
    if sample is None or len(tri) <= sample:
        idx = np.arange(len(tri))
        assert D.violations(m1, tri) == []
    else:
        idx = np.random.default_rng(seed).choice(len(tri), sample, replace=False)
    slack = 1 + 1e-9  # the library decides the bounds in FP64
    for r2, b2 in (D.quality(m1, tri[idx])):
        if R > 0:
            assert r2 <= Fraction(R * R) * Fraction(slack)
        if B > 0:
            assert b2 <= Fraction(B * B) * Fraction(slack)
    assert D.encroached(m1, tri) == []
    a0, a1 = D.area(m0, m0["tri"]), D.area(m1, tri)
    if m0["px"] == 0 and m0["py"] == 0:
        assert a1 == a0
        assert D.segments_covered(m0, m1)
    else:  # images across a periodic seam are rounded
        assert abs(a1 - a0) <= 1e-12 * a0
    return f"nv {m0['nv']} -> {m1['nv']}, nt {m0['nt']} -> {m1['nt']}, {m1['n_iterations']} iterations"


@pytest.mark.parametrize("case", sorted(CASES))
def test_refined_mesh_properties(S, D, case):
    make, R, B = CASES[case]
    m0 = make()
    st, m1 = host_refine(S, m0, R, B)
    assert st == 0
    assert m1["nt"] > m0["nt"]
    check_refined(D, m0, m1, R, B)
    # the same result on a second run (no dependence on the order of elements
    # within a pass is possible here; this checks that nothing else varies)
    st2, m2 = host_refine(S, m0, R, B)
    assert st2 == 0 and np.array_equal(m1["tri"], m2["tri"]) and np.array_equal(m1["x"], m2["x"])


def test_refinement_reaches_the_size_bound_on_a_lattice(S, D):
    """From the two triangles of the unit square, circumradius bound R:
    splitting right isosceles triangles at their hypotenuse midpoints gives
    the regular split-square lattice, where no edge needs a flip."""
    st, m1 = host_refine(S, points_in_box(0, 1.0, 1.0, 0), 0.2, SQRT2)
    assert st == 0 and m1["n_flips"] == 0
    assert m1["nv"] == 25 and m1["nt"] == 32  # the 5 x 5 lattice
    assert sorted(set(m1["x"])) == [0, 0.25, 0.5, 0.75, 1.0]
    check_refined(D, points_in_box(0, 1.0, 1.0, 0), m1, 0.2, SQRT2)


def test_limits_return_the_mesh_so_far(S, D):
    m0 = points_in_box(40, 1.0, 1.0, 1)
    st, m1 = host_refine(S, m0, 0.02, SQRT2, max_vertices=200)
    assert st == 2 and m0["nv"] < m1["nv"] <= 200  # capacity
    assert D.violations(m1, m1["tri"]) == []
    st, m1 = host_refine(S, m0, 0.02, SQRT2, max_iterations=2)
    assert st == 1 and m1["n_iterations"] == 2  # iteration limit
    assert D.violations(m1, m1["tri"]) == []


def morton_keys(m0, x, y):
    """Z-order keys as rd_delaunay_refine documents them: coordinates
    quantised to 32 bits over the period (periodic axis) or the input's
    extent, bits interleaved with x in the even positions."""
    def quant(c, c0, period):
        lo = 0.0 if period > 0 else float(np.min(c0))
        s = 4294967296.0 / (period if period > 0 else float(np.max(c0)) - float(np.min(c0)))
        q = np.clip((np.asarray(c) - lo) * s, 0.0, 4294967295.0)
        return q.astype(np.uint64)

    def spread(v):
        v = v.copy()
        for shift, mask in ((16, 0x0000ffff0000ffff), (8, 0x00ff00ff00ff00ff), (4, 0x0f0f0f0f0f0f0f0f),
                            (2, 0x3333333333333333), (1, 0x5555555555555555)):
            v = (v | (v << np.uint64(shift))) & np.uint64(mask)
        return v

    return spread(quant(x, m0["x"], m0["px"])) | (spread(quant(y, m0["y"], m0["py"])) << np.uint64(1))


def centroids(m):
    """Triangle centroids, corners at their images nearest to corner 0, the
    mean wrapped into the period."""
    t = np.asarray(m["tri"])
    out = []
    for c, per in ((m["x"], m["px"]), (m["y"], m["py"])):
        a = c[t[:, 0]]
        v = [a] + [np.where(c[t[:, k]] - a > 0.5 * per, c[t[:, k]] - per,
                            np.where(c[t[:, k]] - a < -0.5 * per, c[t[:, k]] + per, c[t[:, k]])) if per > 0
                   else c[t[:, k]] for k in (1, 2)]
        g = (v[0] + v[1] + v[2]) / 3.0
        if per > 0:
            g = np.where(g < 0, g + per, g)
            g = np.where(g >= per, g - per, g)
        out.append(g)
    return out


@pytest.mark.parametrize("case", ["random_points", "periodic", "periodic_x_walls_y"])
def test_morton_renumbering(S, D, case):
    """With morton = 1 the refined mesh has the same properties, and its
    vertices and triangles end in non-decreasing Z-order."""
    make, R, B = CASES[case]
    m0 = make()
    st, m1 = host_refine(S, m0, R, B, morton=True)
    assert st == 0
    check_refined(D, m0, m1, R, B, morton=True)
    # ordered by the top 32 bits of the key (a 2^16 x 2^16 grid of cells)
    kv = morton_keys(m0, m1["x"], m1["y"]) >> np.uint64(32)
    assert np.all(kv[1:] >= kv[:-1])
    cx, cy = centroids(m1)
    kt = morton_keys(m0, cx, cy) >> np.uint64(32)
    assert np.all(kt[1:] >= kt[:-1])


def size_field(m0, grid, x, y):
    """The documented size field s at points (x, y): bilinear on the grid's
    nodes (periodic axis: spacing period / n from 0, wrapping; bounded axis:
    n nodes spanning the input's extent)."""
    def axis(v, c0, period, n):
        if period > 0:
            q = np.asarray(v) / (period / n)
            fl = np.floor(q)
            i0 = np.mod(fl.astype(np.int64), n)
            return i0, np.mod(i0 + 1, n), q - fl
        lo, hi = float(np.min(c0)), float(np.max(c0))
        q = np.clip((np.asarray(v) - lo) / ((hi - lo) / (n - 1)), 0, n - 1)
        fl = np.clip(np.floor(q), 0, n - 2)
        return fl.astype(np.int64), fl.astype(np.int64) + 1, q - fl

    x0, x1, wx = axis(x, m0["x"], m0["px"], grid.shape[1])
    y0, y1, wy = axis(y, m0["y"], m0["py"], grid.shape[0])
    a = grid[y0, x0] * (1 - wx) + grid[y0, x1] * wx
    b = grid[y1, x0] * (1 - wx) + grid[y1, x1] * wx
    return a * (1 - wy) + b * wy


def graded_grid(n=9):
    """Scale factors 0.25 along the horizontal mid-line of the domain rising
    linearly to 1 at the top and bottom (n x n nodes)."""
    yy = np.linspace(0.0, 1.0, n)
    s = 0.25 + 1.5 * np.abs(yy - 0.5)
    return np.repeat(s[:, None], n, axis=1)


def check_size_field(D, m0, m1, R, grid):
    """Every triangle's circumradius within R s(centroid) (FP64, slack 1e-9),
    and the mesh denser where s is small."""
    from fractions import Fraction
    tri = np.asarray(m1["tri"])
    x, y = m1["x"], m1["y"]
    cx = (x[tri[:, 0]] + x[tri[:, 1]] + x[tri[:, 2]]) / 3.0
    cy = (y[tri[:, 0]] + y[tri[:, 1]] + y[tri[:, 2]]) / 3.0
    s = size_field(m0, grid, cx, cy)
    for (r2, _), sc in zip(D.quality(m1, tri), s):
        assert r2 <= Fraction(R * R * sc * sc) * Fraction(1 + 1e-9)
    mid = np.abs(cy - 0.5 * (y.max() + y.min())) < 0.1
    edge = np.abs(cy - 0.5 * (y.max() + y.min())) > 0.4
    return mid.sum(), edge.sum()


def test_size_field_grades_the_mesh(S, D):
    """A size field 0.25 on the mid-line rising to 1 at the top and bottom:
    every triangle meets R s(centroid), and the band around the mid-line
    holds far more triangles than equal-area bands at the edges."""
    m0 = points_in_box(20, 1.0, 1.0, 3)
    grid = graded_grid()
    st, m1 = host_refine(S, m0, 0.08, SQRT2, size_grid=grid)
    assert st == 0
    check_refined(D, m0, m1, 0.08, SQRT2)
    n_mid, n_edge = check_size_field(D, m0, m1, 0.08, grid)
    assert n_mid > 4 * n_edge



def test_size_field_on_a_torus(S, D):
    """The size field wraps on periodic axes: every triangle meets R s(centroid)."""
    m0 = wrapped(I.split_square(8, periodic=(True, True), jitter=0.3, seed=5))
    grid = graded_grid(8)
    st, m1 = host_refine(S, m0, 0.08, SQRT2, size_grid=grid)
    assert st == 0
    check_refined(D, m0, m1, 0.08, SQRT2)
    tri = np.asarray(m1["tri"])
    from fractions import Fraction

    def img(v, o):
        return np.where(v - o > 0.5, v - 1.0, np.where(v - o < -0.5, v + 1.0, v))

    x, y = m1["x"], m1["y"]
    cx = np.mod((x[tri[:, 0]] + img(x[tri[:, 1]], x[tri[:, 0]]) + img(x[tri[:, 2]], x[tri[:, 0]])) / 3.0, 1.0)
    cy = np.mod((y[tri[:, 0]] + img(y[tri[:, 1]], y[tri[:, 0]]) + img(y[tri[:, 2]], y[tri[:, 0]])) / 3.0, 1.0)
    s = size_field(m0, grid, cx, cy)
    for (r2, _), sc in zip(D.quality(m1, tri), s):
        assert r2 <= Fraction(0.08 * 0.08 * sc * sc) * Fraction(1 + 1e-9)
