"""GPU (gfx950) parity of librd against the CPU oracle, through the C ABI.

Tolerances, in the max field-normwise relative error
max_i |a_i - b_i| / max_i |b_i| per field, per step from identical inputs,
use the oracle's own sensitivity s(u): how far one oracle step moves when
its input is perturbed by random relative amounts of size u (four draws).
  * FP64: 1e-12, or 3 s(2^-52) where that is larger. s(2^-52) is below
    3.3e-13 for N, LDA and B on smooth states (the bar is then 1e-12); the
    exceptions are the Bmax/Bmin blends, which take one Theta for all four
    equations from a ratio that rounding in one equation can dominate
    (s up to 1.6e-12 on the Kelvin-Helmholtz case), and states with
    triangles at or near rest, where the pivoted solve is ill-conditioned
    (the Sod tube's exact solution at t = 0.1: s ~ 1e-10).
  * FP32 distribution / FP64 accumulation: 2 s(2^-24): the parameter vectors
    enter the triangle algebra rounded to FP32 (relative 2^-24), and the
    algebra's own rounding is of the same order. Measured errors are
    0.11-0.78 s(2^-24) on every per-step case.
Measured errors and bars are printed.
"""
import os

import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def rd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02028_amd import rd as rdmod
    rdmod.lib()
    return rdmod


def err(a, b):
    return max(np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-300) for k in range(4))


def sensitivity(om, W, dt, scheme, time, rel=2.0 ** -52, reps=4, seed=0, ref=None):
    """How far one oracle step moves under random relative input noise."""
    rng = np.random.default_rng(seed)
    if ref is None:
        ref = om.step(W, dt, scheme, time)
    s = 0.0
    for _ in range(reps):
        Wp = W * (1.0 + rel * rng.choice([-1.0, 0.0, 1.0], size=W.shape))
        s = max(s, err(om.step(Wp, dt, scheme, time), ref))
    return s


def tols(om, W, dt, scheme, time, ref=None):
    """(FP64 bar, FP32 bar) for one step of this case."""
    s64 = sensitivity(om, W, dt, scheme, time, 2.0 ** -52, ref=ref)
    s32 = sensitivity(om, W, dt, scheme, time, 2.0 ** -24, ref=ref)
    return max(TOL64, 3.0 * s64), 2.0 * s32


def say(*a):
    print(*a, flush=True)


def gpu_step(rd, m, W, dt, scheme, time, prec, n=1):
    g = rd.Mesh(m)
    g.set_state(W)
    for _ in range(n):
        g.step(dt, scheme, time, prec)
    out = g.get_state()
    g.close()
    return out


CASES = {
    "periodic_random": lambda: (I.split_square(40, diagonal="random", jitter=0.15, seed=1),
                                lambda m: I.random_smooth_state(m, seed=3, amp=0.2)),
    "sod_walls": lambda: (I.split_square(41, periodic=(False, False), bc=("ghost", "wall")), I.ic_sod),
    "kh": lambda: (I.split_square(48), lambda m: I.ic_kelvin_helmholtz(m, seed=1)),
    "quadrants": lambda: (I.split_square(45, periodic=(False, False), diagonal="random", seed=2),
                          lambda m: I.ic_quadrants(m, I.quadrant_states(4))),
    "closed_box": lambda: (I.split_square(23, periodic=(False, False), bc=("wall", "wall")),
                           lambda m: I.random_smooth_state(m, seed=5, amp=0.2)),
    "morton_channel": lambda: (I.split_square(37, periodic=(True, False), bc=("ghost", "wall"),
                                              renumber="morton", rotate_corners=True, seed=7),
                               lambda m: I.random_smooth_state(m, seed=6, amp=0.15)),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("time", [1, 2])
def test_one_step_all_schemes(orc, rd, case, time):
    m, icf = CASES[case]()
    W = icf(m)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    for scheme in range(5):
        ref = om.step(W, dt, scheme, time)
        t64, t32 = tols(om, W, dt, scheme, time, ref=ref)
        say(f"case={case} nt={m['nt']} scheme={scheme} time={time} fp64")
        e64 = err(gpu_step(rd, m, W, dt, scheme, time, rd.FP64), ref)
        say(f"case={case} nt={m['nt']} scheme={scheme} time={time} fp32")
        e32 = err(gpu_step(rd, m, W, dt, scheme, time, rd.FP32_ACC64), ref)
        say(f"  err fp64 {e64:.2e} (tol {t64:.1e}) fp32 {e32:.2e} (tol {t32:.1e})")
        assert e64 <= t64
        assert e32 <= t32


def test_advected_sine_trajectory_n_euler(orc, rd):
    """64x64 periodic advected density wave, N scheme, forward Euler,
    CFL 0.5, 100 steps: per-step parity at states along the oracle's own
    trajectory, and the end state of the full GPU run."""
    m = I.split_square(64)
    W = I.ic_advected_sine(m)
    om = orc.OracleMesh(m)
    states, dts = [W], []
    for n in range(100):
        dts.append(om.max_dt(states[-1], 0.5))
        states.append(om.step(states[-1], dts[-1], orc.N, orc.EULER1))
    g = rd.Mesh(m)
    for n in (0, 33, 66, 99):
        g.set_state(states[n])
        say(f"advected sine step {n}")
        assert abs(g.max_dt(0.5) - dts[n]) <= 1e-14 * dts[n]
        g.step(dts[n], rd.N, rd.EULER1, rd.FP64)
        assert err(g.get_state(), states[n + 1]) <= TOL64
    g.set_state(W)
    for n in range(100):
        g.step(dts[n], rd.N, rd.EULER1, rd.FP64)
    e = err(g.get_state(), states[-1])
    say(f"advected sine 100-step end-state error {e:.2e}")
    assert e <= 1e-12
    g.close()


def test_step_cfl_matches_oracle_trajectory(orc, rd):
    m = I.split_square(33, periodic=(False, False), bc=("ghost", "wall"), diagonal="random", seed=3)
    W = I.ic_quadrants(m, I.quadrant_states(9))
    om = orc.OracleMesh(m)
    ref = W
    for _ in range(10):
        ref = om.step(ref, om.max_dt(ref, 0.4), orc.B, orc.RK2)
    g = rd.Mesh(m)
    g.set_state(W)
    g.step_cfl(10, 0.4, rd.B, rd.RK2, rd.FP64)
    e = err(g.get_state(), ref)
    say(f"step_cfl 10 steps error {e:.2e}")
    assert e <= 1e-12
    g.close()


def test_residual_and_triangle_residual(orc, rd):
    for name in ("periodic_random", "sod_walls", "closed_box"):
        m, icf = CASES[name]()
        W = icf(m)
        om = orc.OracleMesh(m)
        g = rd.Mesh(m)
        g.set_state(W)
        rng = np.random.default_rng(1)
        for scheme in range(5):
            say(f"residual case={name} scheme={scheme}")
            R, phiT = g.residual(scheme, with_phiT=True)
            Ro, phiTo = om.residual(W, scheme, with_phiT=True)
            scale = np.abs(Ro).max()
            noise = 0.0
            for _ in range(3):
                Wp = W * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 0.0, 1.0], size=W.shape))
                noise = max(noise, np.abs(om.residual(Wp, scheme) - Ro).max())
            e = np.abs(R - Ro).max()
            say(f"  residual error {e / scale:.2e}, oracle 1-ulp sensitivity {noise / scale:.2e}")
            assert e <= max(1e-12 * scale, 10 * noise)
            assert np.abs(phiT - phiTo).max() <= 1e-12 * np.abs(phiTo).max()
        g.close()


def test_bitwise_determinism(rd):
    m = I.split_square(129, diagonal="random", seed=4)
    W = I.ic_kelvin_helmholtz(m, seed=4)
    outs = []
    for rep in range(3):
        say(f"determinism rep {rep}")
        g = rd.Mesh(m)
        g.set_state(W)
        g.step_cfl(5, 0.4, rd.B, rd.RK2, rd.FP64)
        g.step_cfl(2, 0.4, rd.B, rd.RK2, rd.FP32_ACC64)
        outs.append(g.get_state())
        g.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec", [0, 1])
def test_uniform_states_preserved_bitwise(rd, prec):
    cases = [(I.split_square(50, diagonal="random", seed=5, jitter=0.2), (1.3, 0.4, -0.7, 0.8)),
             (I.split_square(31, periodic=(False, False), bc=("ghost", "wall")), (0.9, 0.5, 0.0, 1.7)),
             (I.split_square(31, periodic=(False, False), bc=("wall", "wall")), (1.0, 0.0, 0.0, 1.0))]
    for m, prim in cases:
        W = I.ic_uniform(m, *prim)
        for scheme in range(5):
            for time in (1, 2):
                say(f"uniform nt={m['nt']} scheme={scheme} time={time} prec={prec}")
                out = gpu_step(rd, m, W, 1e-3, scheme, time, prec, n=2)
                assert np.array_equal(out, W)


def test_all_ghost_and_tiny_meshes(orc, rd):
    m = I.split_square(2, periodic=(False, False), bc=("ghost", "ghost"))  # every vertex a ghost
    assert m["ghost"].all()
    W = I.ic_quadrants(m, I.quadrant_states(1))
    out = gpu_step(rd, m, W, 1e-3, rd.B, rd.RK2, rd.FP64)
    assert np.array_equal(out, W)
    m = I.split_square(3, periodic=(False, False), bc=("ghost", "ghost"))  # one interior vertex
    W = I.ic_quadrants(m, I.quadrant_states(1))
    om = orc.OracleMesh(m)
    out = gpu_step(rd, m, W, 1e-3, rd.B, rd.RK2, rd.FP64)
    assert err(out, om.step(W, 1e-3, orc.B, orc.RK2)) <= TOL64
    assert np.array_equal(np.delete(out, 4, axis=1), np.delete(W, 4, axis=1))
    m = I.split_square(4, diagonal="random", seed=1)  # 9 vertices, 18 triangles
    W = I.random_smooth_state(m, seed=1)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    for scheme in range(5):
        t64, _ = tols(om, W, dt, scheme, 2)
        assert err(gpu_step(rd, m, W, dt, scheme, 2, rd.FP64), om.step(W, dt, scheme, 2)) <= t64


@pytest.mark.parametrize("tile", [0, 32])
def test_subnormal_momentum_at_rest(orc, rd, tile):
    """A uniform state at rest with one vertex's momentum subnormal (as the
    numerical domain of dependence brings into a quiet region): every blend
    denominator is subnormal and its reciprocal overflows; the step must stay
    finite and match the oracle."""
    for m in (I.split_square(9), I.split_square(9, periodic=(False, False), bc=("ghost", "wall"))):
        W = I.ic_uniform(m, 0.125, 0.0, 0.0, 0.1)
        om = orc.OracleMesh(m)
        for mom in (2.6e-307, 1e-310, 3e-320):
            Wp = W.copy()
            Wp[1, m["nv"] // 2] = mom
            ref = om.step(Wp, 1e-3, orc.B, orc.RK2)
            for prec in (rd.FP64, rd.FP32_ACC64):
                say(f"subnormal momentum {mom} periodic={m['px'] > 0} prec={prec} tile={tile}")
                g = rd.Mesh(m)
                g.tile = tile
                g.set_state(Wp)
                g.step(1e-3, rd.B, rd.RK2, prec)
                g.sync()
                out = g.get_state()
                g.close()
                assert np.isfinite(out).all()
                assert np.abs(out - ref).max() <= 1e-12


def test_device_pointers_and_nonphysical_flag(orc, rd):
    import torch
    m = I.split_square(20)
    W = I.ic_kelvin_helmholtz(m, seed=3)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    g = rd.Mesh(m)
    Wt = torch.from_numpy(W).cuda()
    rd.rd_set_state(g.h, Wt)
    g.step(dt, rd.B, rd.RK2, rd.FP64)
    out = torch.zeros_like(Wt)
    rd.rd_get_state(g.h, out)
    torch.cuda.synchronize()
    assert err(out.cpu().numpy(), om.step(W, dt, orc.B, orc.RK2)) <= TOL64
    R = torch.zeros_like(Wt)
    rd.rd_residual(g.h, rd.B, R)
    torch.cuda.synchronize()
    g.sync()
    # host input with negative pressure is refused
    bad = W.copy()
    bad[3, 7] = 0.1 * 0.5 * (bad[1, 7] ** 2 + bad[2, 7] ** 2) / bad[0, 7]
    with pytest.raises(rd.RDError) as e:
        g.set_state(bad)
    assert e.value.status == rd.RD_ENONPHYS
    # device input is checked on the device and reported by rd_sync
    rd.rd_set_state(g.h, torch.from_numpy(bad).cuda())
    with pytest.raises(rd.RDError) as e:
        g.sync()
    assert e.value.status == rd.RD_ENONPHYS
    g.set_state(W)
    g.sync()
    for args in [(0.0, rd.B, rd.RK2, rd.FP64), (dt, 9, rd.RK2, rd.FP64), (dt, rd.B, 3, rd.FP64),
                 (dt, rd.B, rd.RK2, 5)]:
        with pytest.raises(rd.RDError) as e:
            g.step(*args)
        assert e.value.status == rd.RD_EINVAL
    g.close()


def test_precision_switch(orc, rd):
    m = I.split_square(30, diagonal="random", seed=8)
    W = I.random_smooth_state(m, seed=8, amp=0.2)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    g = rd.Mesh(m)
    g.set_state(W)
    g.step(dt, rd.B, rd.RK2, rd.FP32_ACC64)
    mid = g.get_state()
    g.step(dt, rd.B, rd.RK2, rd.FP64)
    assert err(g.get_state(), om.step(mid, dt, orc.B, orc.RK2)) <= TOL64
    g.close()


# ------------------------------------------------ full-size configurations --

def test_sod_1024_one_step_full_size(orc, rd):
    """1024x1024 Sod tube (2,093,058 triangles), B / RK2 / CFL 0.4: one step
    from the initial state and one from the exact solution at t = 0.1."""
    import exact_riemann as E
    m = I.split_square(1024, periodic=(False, False), bc=("ghost", "wall"))
    om = orc.OracleMesh(m)
    W0 = I.ic_sod(m)
    r, u, p = E.sample(np.unique(m["x"]), 0.1, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    ix = np.searchsorted(np.unique(m["x"]), m["x"])
    W1 = I.prim_to_cons(r[ix], u[ix], 0.0, p[ix])
    for name, W in (("initial", W0), ("exact t=0.1", W1)):
        dt = om.max_dt(W, 0.4)
        ref = om.step(W, dt, orc.B, orc.RK2)
        t64, t32 = tols(om, W, dt, orc.B, orc.RK2, ref=ref)
        say(f"sod 1024 {name} fp64")
        e64 = err(gpu_step(rd, m, W, dt, rd.B, rd.RK2, rd.FP64), ref)
        say(f"sod 1024 {name} fp32")
        e32 = err(gpu_step(rd, m, W, dt, rd.B, rd.RK2, rd.FP32_ACC64), ref)
        say(f"  sod 1024 {name}: fp64 {e64:.2e} (tol {t64:.1e}) fp32 {e32:.2e} (tol {t32:.1e})")
        assert e64 <= t64 and e32 <= t32


@pytest.mark.parametrize("tile", [0, 256])
def test_sod_1024_device_dt_sequence(orc, rd, tile):
    """20 steps with the time step reduced on the device (rd_step_cfl) equal
    20 steps with the oracle's CFL limit of each GPU state passed in from the
    host: at full size every device reduction gives the oracle's dt."""
    m = I.split_square(1024, periodic=(False, False), bc=("ghost", "wall"))
    om = orc.OracleMesh(m)
    W0 = I.ic_sod(m)
    g = rd.Mesh(m)
    g.tile = tile
    g.set_state(W0)
    say(f"sod 1024 device dt tile={tile}")
    g.step_cfl(20, 0.4, rd.B, rd.RK2, rd.FP64)
    a = g.get_state()
    g.set_state(W0)
    W = W0
    for n in range(20):
        dt = om.max_dt(W, 0.4)
        assert abs(g.max_dt(0.4) - dt) <= 1e-14 * dt
        g.step(dt, rd.B, rd.RK2, rd.FP64)
        W = g.get_state()
    g.close()
    e = err(a, W)
    say(f"  device-dt vs host-dt run: {e:.2e}")
    assert e <= 1e-13


def test_kh_2048_one_step_full_size(orc, rd):
    """2048x2048 periodic Kelvin-Helmholtz (8,380,418 triangles), B / RK2,
    the launch configuration the benchmark times."""
    m = I.split_square(2048)
    om = orc.OracleMesh(m)
    W = I.ic_kelvin_helmholtz(m, seed=0)
    dt = om.max_dt(W, 0.4)
    ref = om.step(W, dt, orc.B, orc.RK2)
    t64, t32 = tols(om, W, dt, orc.B, orc.RK2, ref=ref)
    say("kh 2048 fp64")
    g = rd.Mesh(m)
    g.set_state(W)
    assert abs(g.max_dt(0.4) - dt) <= 1e-14 * dt
    g.step_cfl(1, 0.4, rd.B, rd.RK2, rd.FP64)
    e64 = err(g.get_state(), ref)
    say("kh 2048 fp32")
    g.set_state(W)
    g.step_cfl(1, 0.4, rd.B, rd.RK2, rd.FP32_ACC64)
    e32 = err(g.get_state(), ref)
    g.close()
    say(f"  kh 2048: fp64 {e64:.2e} (tol {t64:.1e}) fp32 {e32:.2e} (tol {t32:.1e})")
    assert e64 <= t64 and e32 <= t32


# ------------------------------------------------------------ batches ---

def test_batch_bitwise_equals_single_runs(orc, rd):
    """Independent four-quadrant meshes of uneven size advanced together in
    one captured graph give, mesh by mesh, bitwise the result of each mesh's
    own run, and match the oracle."""
    sides = [17, 33, 9, 40, 24, 3, 50]
    meshes, states = I.batch_problem(seed=3, sides=sides, draw=I.NARROW_QUADRANTS)
    for prec in (rd.FP64, rd.FP32_ACC64):
        singles = []
        for m, W in zip(meshes, states):
            say(f"batch single N={m['N']} prec={prec}")
            g = rd.Mesh(m)
            g.set_state(W)
            g.step_cfl(6, 0.4, rd.B, rd.RK2, prec)
            singles.append(g.get_state())
            g.close()
        gm = [rd.Mesh(m) for m in meshes]
        for g, W in zip(gm, states):
            g.set_state(W)
        b = rd.Batch(gm)
        say(f"batch run prec={prec}")
        b.run(3, 0.4, rd.B, rd.RK2, prec)
        b.run(3, 0.4, rd.B, rd.RK2, prec)   # replays the cached graph
        for g, ref in zip(gm, singles):
            assert np.array_equal(g.get_state(), ref)
        # a member continues on its own after the batch
        gm[3].step_cfl(1, 0.4, rd.B, rd.RK2, prec)
        gm[3].sync()
        b.close()
        for g in gm:
            g.close()
    m, W = meshes[3], states[3]
    om = orc.OracleMesh(m)
    ref = W
    for _ in range(6):
        ref = om.step(ref, om.max_dt(ref, 0.4), orc.B, orc.RK2)
    g = rd.Mesh(m)
    g.set_state(W)
    b = rd.Batch([g])
    b.run(6, 0.4, rd.B, rd.RK2, rd.FP64)
    assert err(g.get_state(), ref) <= 1e-12
    b.close()
    g.close()


def _physical(W, gamma=1.4):
    rho = W[0]
    p = (gamma - 1.0) * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / rho)
    return bool(np.all(np.isfinite(W)) and np.all(rho > 0) and np.all(p > 0))


def test_batch_draw_nonphysical_member_agrees_with_oracle(orc, rd):
    """The batch workload's draw (rho, p ~ U[0.1, 2], |u| <= 1 per quadrant,
    seed 0) includes problems on which the B scheme (not positivity
    preserving) goes non-physical: member 6 (68^2 vertices) does so in its
    6th RK2 step. The GPU and the oracle agree step by step up to that point
    (same CFL dt, 1e-12) and on the step at which the state stops being
    physical; in a batch only that member's latch is set, and every member,
    that one included, is bitwise its own single run."""
    sides = I.batch_sides(0, 256)
    k = 6
    assert sides[k] == 68
    m = I.split_square(sides[k], periodic=(False, False), bc=("ghost", "ghost"))
    W0 = I.ic_quadrants(m, I.quadrant_states(k, **I.BATCH_QUADRANTS))
    om = orc.OracleMesh(m)
    g = rd.Mesh(m)
    g.set_state(W0)
    Wo = W0
    first_o = first_g = None
    for s in range(12):
        dt_o = om.max_dt(Wo, 0.4)
        dt_g = g.max_dt(0.4)
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o
        Wo = om.step(Wo, dt_o, orc.B, orc.RK2)
        g.step(dt_g, rd.B, rd.RK2, rd.FP64)
        Wg = np.zeros_like(W0)
        try:
            g.get_state(Wg)
            ok_g = True
        except rd.RDError as e:
            assert e.status == rd.RD_ENONPHYS
            ok_g = False
        ok_o = _physical(Wo)
        say(f"member {k} step {s + 1}: oracle physical {ok_o}, gpu physical {ok_g}")
        if ok_o and ok_g:
            assert err(Wg, Wo) <= TOL64
        if not ok_o and first_o is None:
            first_o = s
        if not ok_g and first_g is None:
            first_g = s
        if first_o is not None and first_g is not None:
            break
    g.close()
    assert first_o == first_g == 5
    # a batch of three members of the same draw, one of which goes non-physical
    idx = [3, 6, 11]
    ms = [I.split_square(sides[j] if j == 6 else 20 + j, periodic=(False, False), bc=("ghost", "ghost"))
          for j in idx]
    Ws = [I.ic_quadrants(mm, I.quadrant_states(j, **I.BATCH_QUADRANTS)) for j, mm in zip(idx, ms)]
    singles, bad_single = [], []
    for j, mm, W in zip(idx, ms, Ws):
        gg = rd.Mesh(mm)
        gg.set_state(W)
        gg.step_cfl(8, 0.4, rd.B, rd.RK2, rd.FP64)
        out = np.zeros_like(W)
        try:
            gg.get_state(out)
        except rd.RDError:
            bad_single.append(j)
        singles.append(out.view(np.uint64).copy())
        gg.close()
    gm = [rd.Mesh(mm) for mm in ms]
    for gg, W in zip(gm, Ws):
        gg.set_state(W)
    b = rd.Batch(gm)
    say("batch of the draw's members 3, 6, 11")
    b.run(8, 0.4, rd.B, rd.RK2, rd.FP64)
    bad_batch = []
    for j, gg, ref in zip(idx, gm, singles):
        out = np.zeros((4, gg.nv))
        try:
            gg.get_state(out)
        except rd.RDError as e:
            assert e.status == rd.RD_ENONPHYS
            bad_batch.append(j)
        assert np.array_equal(out.view(np.uint64), ref)
    b.close()
    for gg in gm:
        gg.close()
    assert bad_batch == bad_single == [6]


def test_batch_with_periodic_members(orc, rd):
    """Members periodic on both axes (Kelvin-Helmholtz and Fourier-density
    problems of different sizes on the unit square), one periodic on x only
    (a channel with walls) and one bounded four-quadrant member advance
    together in one graph: each is bitwise equal to its own run, and the
    periodic ones match the oracle."""
    ms = [I.split_square(24), I.split_square(33, diagonal="random", seed=2),
          I.split_square(30, periodic=(True, False), bc=("ghost", "wall"), diagonal="random", seed=5),
          I.split_square(40, periodic=(False, False), bc=("ghost", "ghost"))]
    Ws = [I.ic_kelvin_helmholtz(ms[0], seed=1), I.ic_fourier_density(ms[1], seed=0),
          I.random_smooth_state(ms[2], seed=4, amp=0.2),
          I.ic_quadrants(ms[3], I.quadrant_states(4, **I.NARROW_QUADRANTS))]
    for prec in (rd.FP64, rd.FP32_ACC64):
        singles = []
        for m, W in zip(ms, Ws):
            say(f"periodic batch single nt={m['nt']} prec={prec}")
            g = rd.Mesh(m)
            g.set_state(W)
            g.step_cfl(6, 0.4, rd.B, rd.RK2, prec)
            singles.append(g.get_state())
            g.close()
        gm = [rd.Mesh(m) for m in ms]
        for g, W in zip(gm, Ws):
            g.set_state(W)
        b = rd.Batch(gm)
        say(f"periodic batch run prec={prec}")
        b.run(6, 0.4, rd.B, rd.RK2, prec)
        for g, ref in zip(gm, singles):
            assert np.array_equal(g.get_state().view(np.uint64), ref.view(np.uint64))
        b.close()
        for g in gm:
            g.close()
        if prec == rd.FP64:
            # the tiled form: its results do not depend on the tiling, so the
            # batch's own tiles give each member's tiled single run bitwise
            tiled = []
            for m, W in zip(ms, Ws):
                g = rd.Mesh(m)
                g.tile = 64
                g.set_state(W)
                g.step_cfl(6, 0.4, rd.B, rd.RK2, prec)
                tiled.append(g.get_state())
                g.close()
            gm = [rd.Mesh(m) for m in ms]
            for g, W in zip(gm, Ws):
                g.set_state(W)
            b = rd.Batch(gm)
            b.set_tile(128)
            say("periodic batch run, tiles of 128")
            b.run(6, 0.4, rd.B, rd.RK2, prec)
            for g, ref in zip(gm, tiled):
                assert np.array_equal(g.get_state().view(np.uint64), ref.view(np.uint64))
            b.close()
            for g in gm:
                g.close()
            for k in (0, 1, 2):
                om = orc.OracleMesh(ms[k])
                ref = Ws[k]
                for _ in range(6):
                    ref = om.step(ref, om.max_dt(ref, 0.4), orc.B, orc.RK2)
                e = err(singles[k], ref)
                say(f"  member {k} vs oracle {e:.2e}")
                assert e <= TOL64


def test_batch_refuses_mixed_periods_and_empty(rd):
    """One period per axis: members periodic on an axis must share it, and a
    bounded member next to them must be fine enough that unwrapping leaves it
    alone."""
    a = rd.Mesh(I.split_square(16))
    b = rd.Mesh(I.split_square(16, length=2.0))            # period 2 on both axes
    c = rd.Mesh(I.split_square(2, periodic=(False, False)))  # one cell: triangles span the whole unit square
    d = rd.Mesh(I.split_square(8, periodic=(False, False)))  # fine enough
    for members, msg in (([a, b], "share the period"), ([a, c], "too large")):
        with pytest.raises(rd.RDError, match=msg) as e:
            rd.Batch(members)
        assert e.value.status == rd.RD_EINVAL
    rd.Batch([a, d]).close()
    with pytest.raises(rd.RDError):
        rd.rd_batch_create([])
    for g in (a, b, c, d):
        g.close()


# ------------------------------------------------------------- adjoint ---

ADJ_CASES = {
    "periodic_random": lambda: (I.split_square(30, diagonal="random", jitter=0.15, seed=1),
                                lambda m: I.random_smooth_state(m, seed=3, amp=0.2)),
    "kh": lambda: (I.split_square(32), lambda m: I.ic_kelvin_helmholtz(m, seed=1)),
    "ghost_walls": lambda: (I.split_square(21, periodic=(False, False), bc=("ghost", "wall"), diagonal="random",
                                           seed=2), lambda m: I.random_smooth_state(m, seed=5, amp=0.2)),
    "fourier_density": lambda: (I.split_square(33), lambda m: I.ic_fourier_density(m, seed=4)),
}


@pytest.mark.parametrize("case", sorted(ADJ_CASES))
def test_adjoint_dot_product_against_oracle_jvp(orc, rd, case):
    """<lam, J v> from the oracle's exact forward-mode derivative equals
    <J^T lam, v> from rd_adjoint_step, for every scheme and time order."""
    m, icf = ADJ_CASES[case]()
    W = icf(m)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    g = rd.Mesh(m)
    g.set_state(W)
    rng = np.random.default_rng(11)
    for time in (1, 2):
        for scheme in range(5):
            v = rng.normal(size=W.shape) * np.abs(W).mean(axis=1, keepdims=True)
            lam = rng.normal(size=W.shape)
            _, Jv = om.step_jvp(W, v, dt, scheme, time)
            JTl = np.zeros_like(W)
            say(f"adjoint case={case} scheme={scheme} time={time}")
            rd.rd_adjoint_step(g.h, W, dt, scheme, time, lam, JTl)
            a, b = float(np.sum(lam * Jv)), float(np.sum(JTl * v))
            scale = float(np.sum(np.abs(lam * Jv)))
            say(f"  <lam,Jv> {a:.15e}  <J^T lam,v> {b:.15e}  rel {abs(a - b) / scale:.2e}")
            assert abs(a - b) <= 1e-12 * scale
    # the mesh's own state is untouched by the adjoint
    assert np.array_equal(g.get_state(), W)
    g.close()


def test_adjoint_kh_2048_full_size(orc, rd):
    """The adjoint at the benchmark's size and configuration (2048x2048
    periodic Kelvin-Helmholtz, 8,380,418 triangles, FP64 B / RK2, fixed dt):
    <lam, J v> from the oracle's exact forward-mode derivative equals
    <J^T lam, v> from rd_adjoint_step."""
    m = I.split_square(2048)
    W = I.ic_kelvin_helmholtz(m, seed=0)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W, 0.4)
    rng = np.random.default_rng(17)
    v = rng.normal(size=W.shape) * np.abs(W).mean(axis=1, keepdims=True)
    lam = rng.normal(size=W.shape)
    say("adjoint kh 2048: oracle jvp")
    _, Jv = om.step_jvp(W, v, dt, orc.B, orc.RK2)
    say("adjoint kh 2048: gpu adjoint")
    g = rd.Mesh(m)
    g.set_state(W)
    JTl = np.zeros_like(W)
    rd.rd_adjoint_step(g.h, W, dt, rd.B, rd.RK2, lam, JTl)
    g.close()
    a, b = float(np.sum(lam * Jv)), float(np.sum(JTl * v))
    scale = float(np.sum(np.abs(lam * Jv)))
    say(f"  <lam,Jv> {a:.15e}  <J^T lam,v> {b:.15e}  rel {abs(a - b) / scale:.2e}")
    assert abs(a - b) <= 1e-12 * scale


def test_rdstep_autograd_matches_oracle_jvp(orc, rd):
    """torch.autograd through RDStep: <grad of <lam, step(W)>, v> equals
    <lam, J v> from the oracle's exact forward-mode derivative."""
    import torch
    from paper_1705_02028_amd.autograd import RDStep
    m = I.split_square(25, periodic=(True, False), bc=("ghost", "wall"), diagonal="random", seed=3)
    W0 = I.random_smooth_state(m, seed=7, amp=0.2)
    om = orc.OracleMesh(m)
    dt = om.max_dt(W0, 0.4)
    g = rd.Mesh(m)
    rng = np.random.default_rng(3)
    for scheme in (rd.N, rd.B):
        lam = rng.normal(size=W0.shape)
        v = rng.normal(size=W0.shape) * np.abs(W0).mean(axis=1, keepdims=True)
        W = torch.tensor(W0, device="cuda", requires_grad=True)
        out = RDStep.apply(W, g, dt, scheme, rd.RK2)
        (out * torch.tensor(lam, device="cuda")).sum().backward()
        a = float(np.sum(W.grad.cpu().numpy() * v))
        _, Jv = om.step_jvp(W0, v, dt, scheme, orc.RK2)
        b = float(np.sum(lam * Jv))
        scale = float(np.sum(np.abs(lam * Jv)))
        say(f"RDStep scheme={scheme}: {a:.15e} vs {b:.15e}")
        assert abs(a - b) <= 1e-12 * scale
        assert err(out.detach().cpu().numpy(), om.step(W0, dt, scheme, orc.RK2)) <= TOL64
    g.close()


@pytest.mark.parametrize("scheme_name", ["B", "LDA"])
def test_rollout_gradient_checkpointed(orc, rd, scheme_name):
    """Gradient of sum (rho_T - rho_target)^2 with respect to the initial
    density (u, v, p fixed), RK2, fixed dt, 40 steps with checkpoints every
    20: directional derivatives against the oracle's exact forward-mode
    rollout, and (LDA) against central differences of the GPU forward. The B
    blend has |.| kinks wherever a residual component crosses zero, so
    central differences do not converge to its derivative; LDA has none."""
    scheme = getattr(rd, scheme_name)
    import torch
    from paper_1705_02028_amd.autograd import RDRollout, conserved_from_density
    m = I.split_square(33)
    W0 = I.ic_fourier_density(m, seed=0)
    target = I.ic_fourier_density(m, seed=1)[0]
    om = orc.OracleMesh(m)
    dt = om.max_dt(W0, 0.4)
    nsteps = 40
    g = rd.Mesh(m)
    dev = torch.device("cuda")
    rho = torch.tensor(W0[0], dtype=torch.float64, device=dev, requires_grad=True)
    u, v, p = 0.5, 0.3, 1.0
    tgt = torch.tensor(target, dtype=torch.float64, device=dev)

    def loss_of(r):
        W = conserved_from_density(r, u, v, p, m["gamma"])
        WT = RDRollout.apply(W, g, dt, nsteps, scheme, rd.RK2, 20)
        return ((WT[0] - tgt) ** 2).sum()

    L = loss_of(rho)
    L.backward()
    grad = rho.grad.detach().cpu().numpy()
    rng = np.random.default_rng(5)
    for trial in range(2):
        d = rng.normal(size=m["nv"])
        # exact directional derivative through the oracle's rollout
        Wd = np.stack([d, d * u, d * v, 0.5 * d * (u * u + v * v)])
        Wc = W0.copy()
        for _ in range(nsteps):
            Wc, Wd = om.step_jvp(Wc, Wd, dt, scheme, orc.RK2)
        exact = float(np.sum(2.0 * (Wc[0] - target) * Wd[0]))
        got = float(np.dot(grad, d))
        say(f"rollout gradient: <grad,d> {got:.15e} exact {exact:.15e}")
        assert abs(got - exact) <= 1e-10 * abs(exact)
        if scheme == rd.B:
            continue
        eps = 1e-6
        with torch.no_grad():
            dd = torch.tensor(d, dtype=torch.float64, device=dev)
            fd = (loss_of(rho + eps * dd) - loss_of(rho - eps * dd)).item() / (2 * eps)
        say(f"  central difference {fd:.10e}")
        assert abs(fd - got) <= 1e-6 * abs(got)
    g.close()
