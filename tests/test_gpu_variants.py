"""GPU parity of the Bx blend (Section 3.3.3) and of selective lumping
(Section 3.4) against the CPU oracle, through the C ABI, in the two-pass and
the tiled form, per step and over CFL-limited runs, alone and in batches.
Bars as in test_gpu_parity: FP64 max(1e-12, 3 s(2^-52)), FP32_ACC64
2 s(2^-24), s the oracle's own sensitivity on the case.
"""
import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I
from test_gpu_parity import CASES, err, say, tols

pytestmark = pytest.mark.gpu

VCASES = dict(CASES)
VCASES["rect_periodic_y"] = lambda: (I.split_square(30, periodic=(False, True), bc=("ghost", "ghost"), Ny=21,
                                                    ly=2.0, diagonal="random", seed=8),
                                     lambda m: I.random_smooth_state(m, seed=9, amp=0.3))


@pytest.fixture(scope="module")
def rd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02028_amd import rd as rdmod
    rdmod.lib()
    return rdmod


def run(rd, m, W, dt, scheme, time, prec, tile=0, lump=0, n=1, cfl=None):
    g = rd.Mesh(m)
    g.tile = tile
    g.lumping = lump
    assert g.lumping == lump
    g.set_state(W)
    if cfl is None:
        for _ in range(n):
            g.step(dt, scheme, time, prec)
    else:
        g.step_cfl(n, cfl, scheme, time, prec)
    out = g.get_state()
    g.close()
    return out


@pytest.mark.parametrize("case", sorted(VCASES))
@pytest.mark.parametrize("time", [1, 2])
def test_bx_and_selective_lumping_one_step(orc, rd, case, time):
    m, icf = VCASES[case]()
    W = icf(m)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    # Bx with global lumping; every scheme with selective lumping (RK2 only: it
    # does nothing in a forward Euler step)
    combos = [(5, 0)] + ([(s, 1) for s in range(6)] if time == 2 else [])
    for scheme, lump in combos:
        om.set_lumping(bool(lump))
        ref = om.step(W, dt, scheme, time)
        t64, t32 = tols(om, W, dt, scheme, time, ref=ref)
        for tile in (0, 64):
            for prec, bar in ((rd.FP64, t64), (rd.FP32_ACC64, t32)):
                say(f"case={case} nt={m['nt']} scheme={scheme} lump={lump} time={time} tile={tile} prec={prec}")
                e = err(run(rd, m, W, dt, scheme, time, prec, tile, lump), ref)
                say(f"  err {e:.2e} (tol {bar:.1e})")
                assert e <= bar


def test_bx_residual(orc, rd):
    for name in ("kh", "quadrants", "sod_walls"):
        m, icf = CASES[name]()
        W = icf(m)
        om = orc.OracleMesh(m)
        g = rd.Mesh(m)
        g.set_state(W)
        say(f"Bx residual case={name}")
        R = g.residual(rd.BX)
        Ro = om.residual(W, orc.BX)
        e = np.abs(R - Ro).max() / np.abs(Ro).max()
        say(f"  error {e:.2e}")
        assert e <= 1e-12
        g.close()


def test_bx_and_lumping_cfl_runs(orc, rd):
    m = I.split_square(33, periodic=(False, False), bc=("ghost", "wall"), diagonal="random", seed=3)
    W = I.ic_quadrants(m, I.quadrant_states(9))
    om = orc.OracleMesh(m)
    for scheme, lump in ((rd.BX, 0), (rd.B, 1), (rd.BX, 1)):
        om.set_lumping(bool(lump))
        ref = W
        for _ in range(10):
            ref = om.step(ref, om.max_dt(ref, 0.4), scheme, orc.RK2)
        for tile in (0, 128):
            for prec, bar in ((rd.FP64, 1e-12), (rd.FP32_ACC64, 2e-7)):
                say(f"cfl run scheme={scheme} lump={lump} tile={tile} prec={prec}")
                e = err(run(rd, m, W, 0.0, scheme, rd.RK2, prec, tile, lump, n=10, cfl=0.4), ref)
                say(f"  err {e:.2e}")
                assert e <= bar


def test_variants_keep_uniform_states_bitwise(rd):
    m = I.split_square(31, diagonal="random", seed=5, jitter=0.2)
    W = I.ic_uniform(m, 1.3, 0.4, -0.7, 0.8)
    for tile in (0, 64):
        for prec in (rd.FP64, rd.FP32_ACC64):
            for scheme, lump in ((rd.BX, 0), (rd.BX, 1), (rd.B, 1), (rd.N, 1)):
                say(f"uniform scheme={scheme} lump={lump} tile={tile} prec={prec}")
                assert np.array_equal(run(rd, m, W, 1e-3, scheme, rd.RK2, prec, tile, lump, n=2), W)


def test_variants_in_batches(orc, rd):
    """Per-mesh speed ranges and domain sizes: each batch member equals its
    own run bitwise; members with different lumpings are refused."""
    sides = [17, 33, 9, 40, 24]
    meshes, states = I.batch_problem(seed=4, sides=sides, draw=I.NARROW_QUADRANTS)
    for scheme, lump in ((rd.BX, 0), (rd.B, 1), (rd.BX, 1)):
        for tile in (0, 64):
            prec = rd.FP64
            singles = [run(rd, mm, W, 0.0, scheme, rd.RK2, prec, tile, lump, n=5, cfl=0.4)
                       for mm, W in zip(meshes, states)]
            gm = [rd.Mesh(mm) for mm in meshes]
            for g, W in zip(gm, states):
                g.set_state(W)
                g.lumping = lump
            b = rd.Batch(gm)
            b.set_tile(tile)
            say(f"batch scheme={scheme} lump={lump} tile={tile}")
            b.run(5, 0.4, scheme, rd.RK2, prec)
            for g, ref in zip(gm, singles):
                assert np.array_equal(g.get_state(), ref)
            gm[1].lumping = 1 - lump
            with pytest.raises(rd.RDError) as e:
                b.run(1, 0.4, scheme, rd.RK2, prec)
            assert e.value.status == rd.RD_EINVAL
            b.close()
            for g in gm:
                g.close()
    m, W = meshes[3], states[3]
    om = orc.OracleMesh(m)
    ref = W
    for _ in range(5):
        ref = om.step(ref, om.max_dt(ref, 0.4), orc.BX, orc.RK2)
    assert err(run(rd, m, W, 0.0, rd.BX, rd.RK2, rd.FP64, 0, 0, n=5, cfl=0.4), ref) <= 1e-12


def test_adjoint_refuses_bx_and_selective_lumping(rd):
    import torch
    m = I.split_square(20)
    W = I.random_smooth_state(m, seed=1, amp=0.2)
    g = rd.Mesh(m)
    g.set_state(W)
    Wt = torch.from_numpy(W).cuda()
    lam = torch.ones_like(Wt)
    out = torch.empty_like(Wt)
    with pytest.raises(rd.RDError) as e:
        rd.rd_adjoint_step(g.h, Wt, 1e-3, rd.BX, rd.RK2, lam, out)
    assert e.value.status == rd.RD_EUNSUPPORTED
    g.lumping = rd.LUMP_SELECTIVE
    with pytest.raises(rd.RDError) as e:
        rd.rd_adjoint_step(g.h, Wt, 1e-3, rd.B, rd.RK2, lam, out)
    assert e.value.status == rd.RD_EUNSUPPORTED
    rd.rd_adjoint_step(g.h, Wt, 1e-3, rd.B, rd.EULER1, lam, out)  # no stage 2: allowed
    with pytest.raises(rd.RDError) as e:
        g.lumping = 2
    assert e.value.status == rd.RD_EINVAL
    g.close()


def test_bx_and_lumping_kh_2048_full_size(orc, rd):
    """2048x2048 periodic Kelvin-Helmholtz, one CFL step, Bx and B with
    selective lumping, both forms, both precisions."""
    m = I.split_square(2048)
    om = orc.OracleMesh(m)
    W = I.ic_kelvin_helmholtz(m, seed=0)
    dt = om.max_dt(W, 0.4)
    g = rd.Mesh(m)
    for scheme, lump in ((rd.BX, 0), (rd.B, 1)):
        om.set_lumping(bool(lump))
        ref = om.step(W, dt, scheme, orc.RK2)
        t64, t32 = tols(om, W, dt, scheme, orc.RK2, ref=ref)
        g.lumping = lump
        for tile in (0, 256):
            g.tile = tile
            for prec, bar in ((rd.FP64, t64), (rd.FP32_ACC64, t32)):
                say(f"kh 2048 scheme={scheme} lump={lump} tile={tile} prec={prec}")
                g.set_state(W)
                g.step_cfl(1, 0.4, scheme, rd.RK2, prec)
                e = err(g.get_state(), ref)
                say(f"  err {e:.2e} (tol {bar:.1e})")
                assert e <= bar
    g.close()
