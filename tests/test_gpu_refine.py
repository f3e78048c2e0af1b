"""GPU Delaunay refinement (rd_delaunay_refine) against the exact reference
properties (oracle/delaunay.py, via test_refine_cpu.check_refined): valid,
Delaunay, within the size and quality bounds, no encroached segment, area and
segments kept. The GPU passes take their decisions with integer atomics of
fixed priorities and number new elements by prefix sums, so their result
must also equal, bit for bit, a sequential run of the same per-element code
on the CPU (a check that no pass depends on scheduling); at the size of the
paper's mesh-generation test (a uniform periodic mesh of 1.3 million
vertices) the properties are checked exactly on a seeded sample."""
import time

import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I
from test_gpu_parity import say
from test_refine_cpu import CASES, SQRT2, check_refined, host_refine, wrapped

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


@pytest.fixture(scope="module")
def S():
    from test_refine_cpu import build_shim
    return build_shim()


def same(a, b):
    return (a["nv"] == b["nv"] and a["nt"] == b["nt"] and a["n_iterations"] == b["n_iterations"]
            and a["n_flips"] == b["n_flips"] and np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])
            and np.array_equal(a["tri"], b["tri"]))


@pytest.mark.parametrize("morton", [False, True])
@pytest.mark.parametrize("case", sorted(CASES))
def test_refinement_properties_and_host_equality(rd, D, S, case, morton):
    make, R, B = CASES[case]
    m0 = make()
    say(f"refine case={case} nv={m0['nv']} R={R} B={B} morton={morton}")
    m1 = rd.rd_delaunay_refine(m0, R, B, max_vertices=20000, max_triangles=2 * 20000 + m0["nt"], morton=morton)
    say("  " + check_refined(D, m0, m1, R, B, morton=morton))
    st, h = host_refine(S, m0, R, B, morton=morton)
    assert st == 0 and same(m1, h)


@pytest.mark.parametrize("morton", [False, True])
def test_medium_periodic_mesh_equals_host_run(rd, D, S, morton):
    m0 = wrapped(I.split_square(16, periodic=(True, True), jitter=0.3, seed=9))
    R = 0.004
    say(f"refine periodic 16^2 R={R} morton={morton}")
    t0 = time.perf_counter()
    m1 = rd.rd_delaunay_refine(m0, R, SQRT2, max_vertices=200000, morton=morton)
    el = time.perf_counter() - t0
    say(f"  {m1['nv']} vertices, {m1['nt']} triangles, {m1['n_iterations']} iterations, "
        f"{m1['n_flips']} flips, {el:.2f} s")
    st, h = host_refine(S, m0, R, SQRT2, max_vertices=200000, morton=morton)
    assert st == 0 and same(m1, h)
    say("  " + check_refined(D, m0, m1, R, SQRT2, sample=3000, seed=1, morton=morton))


@pytest.mark.parametrize("morton", [False, True])
def test_paper_size_periodic_mesh(rd, D, morton):
    """A uniform periodic mesh of about 1.3 million vertices (the paper's
    mesh-generation test), refined from a jittered 32 x 32 lattice with the
    quality bound sqrt 2 and a circumradius bound."""
    m0 = wrapped(I.split_square(32, periodic=(True, True), jitter=0.3, seed=10))
    R = 7.3e-4
    rd.rd_delaunay_refine(m0, 0.05, SQRT2)  # first call: module load, allocator
    t0 = time.perf_counter()
    m1 = rd.rd_delaunay_refine(m0, R, SQRT2, max_vertices=1600000, morton=morton)
    el = time.perf_counter() - t0
    say(f"refine periodic (morton={morton}) to {m1['nv']} vertices, {m1['nt']} triangles: "
        f"{m1['n_iterations']} iterations, {m1['n_flips']} flips, {el:.2f} s")
    assert same(m1, rd.rd_delaunay_refine(m0, R, SQRT2, max_vertices=1600000, morton=morton))  # run to run
    assert 1.1e6 < m1["nv"] < 1.6e6 and m1["nt"] == 2 * m1["nv"]  # a torus: nt = 2 nv
    tri = m1["tri"]
    idx = np.random.default_rng(2).choice(len(tri), 1500, replace=False)
    assert D.violations_at(m1, tri, idx) == []
    from fractions import Fraction
    for r2, b2 in D.quality(m1, tri[idx]):
        assert r2 <= Fraction(R * R) * Fraction(1 + 1e-9) and b2 <= Fraction(2) * Fraction(1 + 1e-9)
    # whole-mesh checks in FP64: positive areas summing to the torus's area
    x, y = m1["x"], m1["y"]

    def img(v, o):
        return np.where(v - o > 0.5, v - 1.0, np.where(v - o < -0.5, v + 1.0, v))

    ax, ay = x[tri[:, 0]], y[tri[:, 0]]
    bx, by = img(x[tri[:, 1]], ax), img(y[tri[:, 1]], ay)
    cx, cy = img(x[tri[:, 2]], ax), img(y[tri[:, 2]], ay)
    det = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    assert det.min() > 0 and abs(det.sum() / 2 - 1.0) < 1e-9
    D.neighbours(tri)  # no edge in three triangles


def test_capacity_limit_returns_a_valid_mesh(rd, D):
    from test_refine_cpu import points_in_box
    m0 = points_in_box(40, 1.0, 1.0, 1)
    with pytest.raises(rd.RDError) as e:
        rd.rd_delaunay_refine(m0, 0.02, SQRT2, max_vertices=200)
    assert e.value.status == rd.RD_ENOMEM


def test_refined_mesh_runs_the_solver(rd):
    """A refined periodic mesh is a valid input of the flow solver: a uniform
    state stays uniform."""
    m0 = wrapped(I.split_square(8, periodic=(True, True), jitter=0.3, seed=11))
    m1 = rd.rd_delaunay_refine(m0, 0.02, SQRT2)
    m = {"x": m1["x"], "y": m1["y"], "tri": m1["tri"], "px": 1.0, "py": 1.0, "nv": m1["nv"], "nt": m1["nt"],
         "gamma": 1.4, "ghost": np.zeros(m1["nv"], dtype=np.uint8), "wall": np.zeros((0, 2), dtype=np.int32)}
    rd.rd_mesh_validate(m)
    g = rd.Mesh(m)
    W = I.ic_uniform(m, 1.2, 0.3, -0.1, 0.9)
    g.set_state(W)
    g.step_cfl(5, 0.4, rd.B, rd.RK2, rd.FP64)
    assert np.allclose(g.get_state(), W, rtol=0, atol=1e-12)
    g.close()


def test_graded_meshes(rd, D, S):
    """A spatially varying size bound (Section 2): the GPU's graded meshes
    equal the sequential host run, meet R s(centroid) everywhere, are
    denser where s is small, and a periodic one carries a Kelvin-Helmholtz
    flow (finer along the shear layers) through a few solver steps."""
    from test_refine_cpu import check_size_field, graded_grid, points_in_box
    m0 = points_in_box(20, 1.0, 1.0, 3)
    grid = graded_grid()
    m1 = rd.rd_delaunay_refine(m0, 0.02, SQRT2, size_grid=grid, max_vertices=100000)
    st, h = host_refine(S, m0, 0.02, SQRT2, max_vertices=100000, size_grid=grid)
    assert st == 0 and same(m1, h)
    n_mid, n_edge = check_size_field(D, m0, m1, 0.02, grid)
    say(f"graded square: {m1['nv']} vertices; {n_mid} triangles near the mid-line, {n_edge} at the edges")
    assert n_mid > 4 * n_edge
    # periodic: fine (s = 0.25) at the two shear layers y = 1/4, 3/4, coarse between
    t0 = wrapped(I.split_square(8, periodic=(True, True), jitter=0.3, seed=14))
    yy = np.arange(16) / 16.0
    s = 0.25 + 3.0 * np.minimum(np.abs(yy - 0.25), np.abs(yy - 0.75))
    tgrid = np.repeat(s[:, None], 4, axis=1)
    t1 = rd.rd_delaunay_refine(t0, 0.02, SQRT2, size_grid=tgrid, morton=True)
    st, h = host_refine(S, t0, 0.02, SQRT2, max_vertices=200000, size_grid=tgrid, morton=True)
    assert st == 0 and same(t1, h)
    m = {"x": t1["x"], "y": t1["y"], "tri": t1["tri"], "px": 1.0, "py": 1.0, "nv": t1["nv"], "nt": t1["nt"],
         "gamma": 1.4}
    rd.rd_mesh_validate(m)
    g = rd.Mesh(m)
    W = I.ic_kelvin_helmholtz(m, seed=15)
    g.set_state(W)
    g.step_cfl(20, 0.4, rd.B, rd.RK2, rd.FP64)
    g.sync()
    out = g.get_state()
    assert np.all(np.isfinite(out)) and out[0].min() > 0
    say(f"graded torus: {t1['nv']} vertices, 20 B/RK2 steps of Kelvin-Helmholtz, min rho {out[0].min():.3f}")
    g.close()
