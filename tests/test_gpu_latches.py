"""State bookkeeping around the calls that run steps on scratch state
(rd_tune, batches, rd_adjoint_step), and the adjoint's latched conditions,
through the C ABI on the GPU."""
import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02028_amd import rd as rdmod
    rdmod.lib()
    return rdmod


def say(*a):
    print(*a, flush=True)


def fresh_dt(rd, m, W, cfl):
    g = rd.Mesh(m)
    g.set_state(W)
    dt = g.max_dt(cfl)
    g.close()
    return dt


@pytest.mark.parametrize("prec_name", ["FP64", "FP32_ACC64"])
def test_max_dt_after_tune(rd, prec_name):
    """rd_tune runs timed steps on the mesh and puts its state back; the CFL
    limit afterwards is the one of that state, not of the last timed step."""
    m = I.split_square(40, diagonal="random", seed=2)
    W = I.ic_kelvin_helmholtz(m, seed=3)
    ref = fresh_dt(rd, m, W, 0.4)
    g = rd.Mesh(m)
    g.set_state(W)
    say(f"max_dt after tune {prec_name}")
    g.tune(0.4, rd.B, rd.RK2, getattr(rd, prec_name), n_steps=3, candidates=[0, 64])
    assert g.max_dt(0.4) == ref
    assert np.array_equal(g.get_state(), W)
    g.close()


def test_max_dt_after_batch_run(rd):
    """A batch run copies new states into its members; their CFL limits
    follow those states."""
    ms = [I.split_square(n, periodic=(False, False)) for n in (17, 23)]
    Ws = [I.ic_quadrants(m, I.quadrant_states(s)) for s, m in enumerate(ms)]
    gs = [rd.Mesh(m) for m in ms]
    for g, W in zip(gs, Ws):
        g.set_state(W)
        g.max_dt(0.4)
    b = rd.Batch(gs)
    say("max_dt after batch run")
    b.run(5, 0.4, rd.B, rd.RK2, rd.FP64)
    for g, m in zip(gs, ms):
        W = g.get_state()
        assert g.max_dt(0.4) == fresh_dt(rd, m, W, 0.4)
    b.close()
    for g in gs:
        g.close()


def test_adjoint_leaves_mesh_bookkeeping(rd):
    """rd_adjoint_step recomputes a step from another state W_n: the mesh's
    own state, CFL limit and non-physical latch are unchanged."""
    m = I.split_square(33)
    W = I.ic_fourier_density(m, seed=0)
    Wn = I.ic_fourier_density(m, seed=5, u=-0.4, v=0.6, p=2.0)
    ref = fresh_dt(rd, m, W, 0.4)
    g = rd.Mesh(m)
    g.set_state(W)
    lam = np.random.default_rng(0).normal(size=W.shape)
    out = np.zeros_like(W)
    say("adjoint then max_dt")
    rd.rd_adjoint_step(g.h, Wn, 1e-3, rd.B, rd.RK2, lam, out)
    assert np.all(np.isfinite(out))
    assert g.max_dt(0.4) == ref
    assert np.array_equal(g.get_state(), W)
    g.sync()
    g.close()


def test_adjoint_nonphysical_input_is_reported(rd):
    """A non-physical W_n is latched by the adjoint's own flag: the host call
    returns RD_ENONPHYS, the device call reports it at rd_sync, and the mesh
    (whose own state is fine) still steps and reads back."""
    import torch
    m = I.split_square(17)
    W = I.ic_fourier_density(m, seed=0)
    bad = W.copy()
    bad[3, 7] = 0.1 * bad[3, 7] - 10.0  # negative pressure at one vertex
    g = rd.Mesh(m)
    g.set_state(W)
    lam = np.ones_like(W)
    out = np.zeros_like(W)
    say("adjoint non-physical, host path")
    with pytest.raises(rd.RDError) as e:
        rd.rd_adjoint_step(g.h, bad, 1e-3, rd.B, rd.RK2, lam, out)
    assert e.value.status == rd.RD_ENONPHYS
    g.sync()  # reported once, then cleared
    say("adjoint non-physical, device path")
    dev = torch.device("cuda")
    tb, tl = torch.tensor(bad, device=dev), torch.tensor(lam, device=dev)
    to = torch.empty_like(tl)
    rd.rd_adjoint_step(g.h, tb, 1e-3, rd.B, rd.RK2, tl, to)
    with pytest.raises(rd.RDError) as e:
        g.sync()
    assert e.value.status == rd.RD_ENONPHYS
    g.sync()
    assert np.array_equal(g.get_state(), W)
    g.step(1e-3, rd.B, rd.RK2, rd.FP64)
    g.get_state()
    g.close()


def test_adjoint_stagnant_triangle_is_reported(rd):
    """At exact rest A = sum K_i^+ is singular (its density column vanishes,
    Section 3.3.1) and the solve skips a column; the adjoint, which needs A's
    inverse, reports RD_EUNSUPPORTED instead of returning a wrong gradient.
    A flow that is at rest only in part of the domain is reported too; a
    moving flow is not."""
    m = I.split_square(17, periodic=(False, False), bc=("ghost", "wall"))
    g = rd.Mesh(m)
    lam = np.random.default_rng(1).normal(size=(4, m["nv"]))
    out = np.zeros_like(lam)
    for name, W in (("rest", I.ic_uniform(m, 1.0, 0.0, 0.0, 1.0)), ("sod", I.ic_sod(m))):
        g.set_state(W)
        for time in (rd.EULER1, rd.RK2):
            say(f"adjoint stagnant {name} time={time}")
            with pytest.raises(rd.RDError) as e:
                rd.rd_adjoint_step(g.h, W, 1e-3, rd.N, time, lam, out)
            assert e.value.status == rd.RD_EUNSUPPORTED
            g.sync()
    W = I.random_smooth_state(m, seed=2, amp=0.1)
    g.set_state(W)
    say("adjoint moving flow")
    rd.rd_adjoint_step(g.h, W, 1e-3, rd.B, rd.RK2, lam, out)
    g.sync()
    g.close()
