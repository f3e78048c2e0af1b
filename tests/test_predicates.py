"""Exact in-circle predicate of the Delaunay flips (rd_predicates.h), on the
CPU: the FP64 filter and the expansion-arithmetic evaluation against exact
rational arithmetic (Python fractions hold every double exactly), on random,
exactly cocircular, one-ulp-perturbed and badly scaled inputs."""
import ctypes as C
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def P():
    out = os.path.join(tempfile.mkdtemp(prefix="pred_"), "libpred.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                    "-Wno-unknown-pragmas", "-I", os.path.join(ROOT, "paper_1705_02028_amd", "csrc"),
                    os.path.join(HERE, "cpp", "predicates_shim.cpp"), "-o", out], check=True)
    L = C.CDLL(out)
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    for n in ("rdp_incircle_filter", "rdp_incircle_exact"):
        getattr(L, n).argtypes = [dp, dp, dp, dp]
        getattr(L, n).restype = C.c_int
    L.rdp_orient.argtypes = [dp, dp, dp]
    L.rdp_orient.restype = C.c_int
    L.rdp_product4.argtypes = [C.c_double] * 4 + [dp]
    L.rdp_product4.restype = C.c_int
    return L


def exact_incircle(a, b, c, d):
    """Sign of the in-circle determinant in exact rationals (the definition)."""
    F = [tuple(Fraction(float(v)) for v in p) for p in (a, b, c, d)]
    (ax, ay), (bx, by), (cx, cy), (dx, dy) = F
    rows = [(px - dx, py - dy) for px, py in ((ax, ay), (bx, by), (cx, cy))]
    m = [(u, v, u * u + v * v) for u, v in rows]
    det = (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
           - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
           + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    return (det > 0) - (det < 0)


def call(L, name, pts):
    return getattr(L, name)(*[np.ascontiguousarray(p, dtype=np.float64) for p in pts])


def check(L, pts):
    want = exact_incircle(*pts)
    assert call(L, "rdp_incircle_exact", pts) == want
    f = call(L, "rdp_incircle_filter", pts)
    assert f == 0 or f == want
    return want, f


def test_expansion_product_is_exact(P):
    rng = np.random.default_rng(0)
    out = np.zeros(16)
    for _ in range(2000):
        v = rng.normal(size=4) * np.exp2(rng.integers(-40, 40, size=4))
        n = P.rdp_product4(*v, out)
        want = Fraction(v[0]) * Fraction(v[1]) * Fraction(v[2]) * Fraction(v[3])
        assert sum(Fraction(x) for x in out[:n]) == want
        mags = np.abs(out[:n])
        assert np.all(mags[:-1] < mags[1:]) and np.all(out[:n] != 0.0)   # increasing, no zeros kept


def test_random_points(P):
    rng = np.random.default_rng(1)
    certain = 0
    for _ in range(3000):
        pts = rng.uniform(-1, 1, size=(4, 2)) * np.exp2(rng.integers(-20, 20))
        _, f = check(P, pts)
        certain += f != 0
    assert certain > 2900   # the filter decides almost every random case


def test_exactly_cocircular_points(P):
    # integer points on x^2 + y^2 = 25 and 65^2, scaled by powers of two and shifted
    circle5 = [(3, 4), (4, 3), (5, 0), (0, 5), (-3, 4), (-4, -3), (0, -5), (3, -4)]
    circle65 = [(16, 63), (25, 60), (33, 56), (39, 52), (52, 39), (56, 33), (60, 25), (63, 16), (65, 0)]
    rng = np.random.default_rng(2)
    for circ in (circle5, circle65):
        for _ in range(200):
            idx = rng.choice(len(circ), size=4, replace=False)
            s = float(np.exp2(rng.integers(-30, 5)))
            off = float(rng.integers(-1000, 1000)) * s
            pts = [(circ[i][0] * s + off, circ[i][1] * s - off) for i in idx]
            want, f = check(P, pts)
            assert want == 0 and f == 0


def test_one_ulp_perturbations_of_cocircular_points(P):
    # shifted so that no coordinate is 0: one ulp of 0 is subnormal, and
    # expansion arithmetic is exact only while no product underflows
    base = [(3.0 + 8, 4.0 + 8), (-4.0 + 8, 3.0 + 8), (0.0 + 8, -5.0 + 8), (5.0 + 8, 0.0 + 8)]
    seen = set()
    for k in range(4):
        for axis in range(2):
            for direction in (-np.inf, np.inf):
                pts = [list(p) for p in base]
                pts[k][axis] = np.nextafter(pts[k][axis], direction)
                want, f = check(P, pts)
                assert f == 0      # within the filter's bound: decided exactly
                seen.add(want)
    assert seen == {-1, 1}


def test_inexact_coordinate_differences(P):
    """Differences that do not fit one double (tiny next to large values):
    the exact path carries their rounding errors as second terms."""
    rng = np.random.default_rng(3)
    for _ in range(500):
        big = 1.0 + rng.integers(0, 2 ** 20) * 2.0 ** -20
        pts = [(big + rng.normal() * 1e-17, rng.normal() * 1e-18) for _ in range(3)]
        pts.append((rng.normal() * 1e-19, big))
        check(P, pts)
    # nearly cocircular, far from the origin, with tiny offsets
    for _ in range(500):
        th = rng.uniform(0, 2 * np.pi, size=4)
        pts = [(1e6 + np.cos(t), -1e6 + np.sin(t)) for t in th]
        check(P, pts)


def test_split_square_cells(P):
    """The four corners of a cell of the split-square mesh (coordinates i h,
    h = 1/(N - 1) rounded): cocircular up to the rounding of i h."""
    for N in (5, 64, 1024, 2048):
        h = 1.0 / (N - 1)
        for i in (0, 1, N // 3, N - 2):
            a, b, c, d = (i * h, i * h), ((i + 1) * h, i * h), ((i + 1) * h, (i + 1) * h), (i * h, (i + 1) * h)
            check(P, [a, b, c, d])


def exact_orient(a, b, c):
    (ax, ay), (bx, by), (cx, cy) = [tuple(Fraction(float(v)) for v in p) for p in (a, b, c)]
    det = (ax - cx) * (by - cy) - (ay - cy) * (bx - cx)
    return (det > 0) - (det < 0)


def test_orientation(P):
    rng = np.random.default_rng(4)
    cases = []
    for _ in range(2000):
        cases.append(rng.uniform(-1, 1, size=(3, 2)) * np.exp2(rng.integers(-20, 20)))
    # collinear points on lines through exactly representable points, and one-ulp moves off them
    for _ in range(500):
        p0 = rng.integers(-1000, 1000, size=2).astype(float)
        dvec = rng.integers(-50, 50, size=2).astype(float)
        k1, k2 = rng.integers(-20, 20, size=2)
        pts = [p0, p0 + k1 * dvec, p0 + k2 * dvec]
        cases.append(np.array(pts))
        moved = np.array(pts)
        moved[2, rng.integers(0, 2)] = np.nextafter(moved[2, rng.integers(0, 2)], np.inf)
        cases.append(moved)
    # nearly collinear with inexact differences
    for _ in range(500):
        t = rng.uniform(0, 1, size=3)
        cases.append(np.array([(0.1 + 0.3 * u, 0.7 - 0.2 * u) for u in t]))
    zero = 0
    for pts in cases:
        want = exact_orient(*pts)
        zero += want == 0
        assert P.rdp_orient(*[np.ascontiguousarray(p, dtype=np.float64) for p in pts]) == want
    assert zero > 100
