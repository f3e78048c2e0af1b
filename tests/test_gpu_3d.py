"""The three-dimensional GPU path (rd3_*) against the three-dimensional
oracle (oracle/rd3_oracle.cpp) on seeded periodic boxes of tetrahedra: one
step of every scheme with forward Euler and RK2, the CFL limit, runs of
CFL-limited steps, and (at the benchmark's size, where the oracle is too
slow to run whole) uniform-state steadiness and conservation. Bar: FP64,
maximum error relative to each component's scale <= 1e-12 for one step."""
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
def O():
    import oracle3
    oracle3.build(force=False)
    return oracle3


def rel_err(a, b):
    scale = np.abs(b).max(axis=1, keepdims=True)
    return float((np.abs(a - b) / scale).max())


MESHES = {
    "periodic_jitter": lambda: I.cube_tets(4, jitter=0.2, seed=1),
    "periodic_morton": lambda: I.cube_tets(5, jitter=0.15, seed=2, renumber="morton"),
    "bounded_z": lambda: I.cube_tets(4, periodic=(True, True, False), jitter=0.2, seed=3),
}
SCHEMES = [("N", 0), ("LDA", 1), ("B", 2), ("BMAX", 3), ("BMIN", 4)]


@pytest.mark.parametrize("mesh", sorted(MESHES))
def test_one_step_matches_the_oracle(rd, O, mesh):
    m = MESHES[mesh]()
    W = I.ic3_random_smooth(m, seed=7)
    om = O.OracleMesh3(m)
    g = rd.Mesh3(m)
    g.set_state(W)
    dt = om.max_dt(W, 0.4)
    assert g.max_dt(0.4) == pytest.approx(dt, rel=1e-13)
    worst = 0.0
    for name, s in SCHEMES:
        for time in (rd.EULER1, rd.RK2):
            g.set_state(W)
            g.step(dt, s, time)
            got = g.get_state()
            ref = om.step(W, dt, s, time)
            e = rel_err(got, ref)
            worst = max(worst, e)
            assert e <= 1e-12, (name, time, e)
    say(f"3d {mesh}: nt={m['nt']} worst one-step error {worst:.2e}")
    g.close()


def test_cfl_steps_match_the_oracle(rd, O):
    m = I.cube_tets(6, jitter=0.2, seed=4)
    W = I.ic3_kelvin_helmholtz(m, seed=5)
    om = O.OracleMesh3(m)
    g = rd.Mesh3(m)
    g.set_state(W)
    g.step_cfl(10, 0.4, rd.B, rd.RK2)
    got = g.get_state()
    ref = W
    for _ in range(10):
        ref = om.step(ref, om.max_dt(ref, 0.4), O.B, O.RK2)
    e = rel_err(got, ref)
    say(f"3d KH 6^3 cells, 10 CFL steps B/RK2: {e:.2e}")
    assert e <= 1e-12
    g.close()


def test_medium_box_matches_the_oracle(rd, O):
    m = I.cube_tets(16, jitter=0.2, seed=6, renumber="morton")
    W = I.ic3_kelvin_helmholtz(m, seed=8)
    om = O.OracleMesh3(m)
    dt = om.max_dt(W, 0.4)
    g = rd.Mesh3(m)
    g.set_state(W)
    g.step(dt, rd.B, rd.RK2)
    e = rel_err(g.get_state(), om.step(W, dt, O.B, O.RK2))
    say(f"3d KH 16^3 cells ({m['nt']} tetrahedra), one B/RK2 step: {e:.2e}")
    assert e <= 1e-12
    g.close()


def test_benchmark_size_properties(rd):
    """128^3 cells (12.6 M tetrahedra): a uniform state stays uniform and
    the Kelvin-Helmholtz state keeps its totals (periodic box)."""
    m = I.cube_tets(128, renumber="morton")
    g = rd.Mesh3(m)
    U = I.ic3_uniform(m, 1.2, 0.3, -0.2, 0.1, 0.9)
    g.set_state(U)
    g.step_cfl(2, 0.4, rd.B, rd.RK2)
    assert np.abs(g.get_state() - U).max() <= 1e-13
    W = I.ic3_kelvin_helmholtz(m, seed=9)
    g.set_state(W)
    g.step_cfl(2, 0.4, rd.B, rd.RK2)
    got = g.get_state()
    h3 = (1.0 / 128) ** 3  # every vertex volume of the regular box
    tot0, tot1 = W.sum(axis=1) * h3, got.sum(axis=1) * h3
    assert np.abs(tot1 - tot0).max() <= 1e-12 * np.abs(tot0).max()
    assert np.all(got[0] > 0)
    say(f"3d 128^3: {m['nt']} tetrahedra, totals drift {np.abs(tot1 - tot0).max():.2e}")
    g.close()


def test_fluid_at_rest_singular_sum(rd, O):
    """With zero velocity everywhere the sum of K^+ over a tetrahedron is
    singular (each corner's K^+ has rank one); the pivoted solve skips the
    empty column on both sides and the parts agree."""
    m = I.cube_tets(5, jitter=0.2, seed=10)
    rng = np.random.default_rng(11)
    W = I.prim_to_cons3(1.0 + 0.1 * rng.random(m["nv"]), 0.0, 0.0, 0.0, 1.0 + 0.1 * rng.random(m["nv"]))
    om = O.OracleMesh3(m)
    dt = om.max_dt(W, 0.4)
    g = rd.Mesh3(m)
    for name, s in SCHEMES:
        for time in (rd.EULER1, rd.RK2):
            g.set_state(W)
            g.step(dt, s, time)
            e = rel_err(g.get_state(), om.step(W, dt, s, time))
            assert e <= 1e-12, (name, time, e)
    g.close()


def test_nonphysical_latch(rd):
    """A time step far beyond the CFL limit drives the density negative
    somewhere: rd3_sync reports RD_ENONPHYS until the next rd3_set_state."""
    m = I.cube_tets(6, jitter=0.2, seed=12)
    W = I.ic3_kelvin_helmholtz(m, seed=13)
    g = rd.Mesh3(m)
    g.set_state(W)
    dt = g.max_dt(0.4)
    g.step(dt, rd.B, rd.RK2)
    g.sync()  # a normal step is fine
    for _ in range(3):
        g.step(200 * dt, rd.N, rd.EULER1)
    with pytest.raises(rd.RDError) as e:
        g.sync()
    assert e.value.status == rd.RD_ENONPHYS
    g.set_state(W)
    g.sync()
    g.close()
