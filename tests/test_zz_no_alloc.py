"""rd_adjoint_step_noalloc (the adjoint of one step on a fixed per-GPU
workspace, calling no allocator) against rd_adjoint_step, through the C ABI:
two calls in a row, the second on a smaller mesh, each equal bit for bit to
the allocating entry point on the same inputs and matching the oracle's
forward-mode derivative; the latches are cleared on every call; a mesh too
large for the workspace is refused."""
import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def rd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1705_02028_amd import rd as rdmod
    rdmod.lib()
    return rdmod


CASES = [
    # larger first, then smaller: the second call reuses the workspace the first filled
    ("walls_ghosts_181", lambda: I.split_square(181, periodic=(True, False), bc=("ghost", "wall"),
                                                diagonal="random", seed=4)),
    ("periodic_40", lambda: I.split_square(40, diagonal="random", jitter=0.1, seed=5)),
]


def test_noalloc_adjoint_equals_allocating_adjoint(rd, orc):
    import torch
    dev = torch.device("cuda")
    flags = torch.full((2,), 7, dtype=torch.int32, device=dev)
    rng = np.random.default_rng(9)
    for name, make in CASES:
        m = make()
        W = I.random_smooth_state(m, seed=6, amp=0.2)
        om = orc.OracleMesh(m)
        dt = om.max_dt(W, 0.4)
        g = rd.Mesh(m)
        g.set_state(W)
        for scheme, time in ((rd.B, rd.RK2), (rd.N, rd.EULER1), (rd.LDA, rd.RK2)):
            lam = rng.normal(size=W.shape)
            v = rng.normal(size=W.shape) * np.abs(W).mean(axis=1, keepdims=True)
            tW, tl = torch.tensor(W, device=dev), torch.tensor(lam, device=dev)
            ref, got = torch.empty_like(tl), torch.full_like(tl, np.nan)
            say(f"noalloc case={name} nv={m['nv']} scheme={scheme} time={time}")
            rd.rd_adjoint_step(g.h, tW, dt, scheme, time, tl, ref)
            g.sync()
            rd.rd_adjoint_step_noalloc(g.h, tW, dt, scheme, time, tl, got, flags)
            torch.cuda.synchronize()
            assert flags.cpu().tolist() == [0, 0]
            r, o = ref.cpu().numpy(), got.cpu().numpy()
            assert np.array_equal(r.view(np.uint64), o.view(np.uint64))
            _, Jv = om.step_jvp(W, v, dt, scheme, time)
            a, b = float(np.sum(lam * Jv)), float(np.sum(o * v))
            say(f"  <lam,Jv> {a:.15e} <J^T lam,v> {b:.15e}")
            assert abs(a - b) <= 1e-12 * float(np.sum(np.abs(lam * Jv)))
        # the mesh's own state is untouched
        assert np.array_equal(g.get_state(), W)
        g.close()


def test_noalloc_latches_and_limits(rd):
    import torch
    dev = torch.device("cuda")
    m = I.split_square(17, periodic=(False, False), bc=("ghost", "wall"))
    g = rd.Mesh(m)
    lam = torch.tensor(np.random.default_rng(1).normal(size=(4, m["nv"])), device=dev)
    out = torch.empty_like(lam)
    flags = torch.zeros(2, dtype=torch.int32, device=dev)
    say("noalloc at rest: skipped column latched")
    rest = torch.tensor(I.ic_uniform(m, 1.0, 0.0, 0.0, 1.0), device=dev)
    rd.rd_adjoint_step_noalloc(g.h, rest, 1e-3, rd.N, rd.RK2, lam, out, flags)
    torch.cuda.synchronize()
    assert flags.cpu().tolist() == [0, 1]
    say("noalloc non-physical input latched")
    bad = I.random_smooth_state(m, seed=2, amp=0.1)
    bad[3, 7] = 0.1 * bad[3, 7] - 10.0
    rd.rd_adjoint_step_noalloc(g.h, torch.tensor(bad, device=dev), 1e-3, rd.B, rd.RK2, lam, out, flags)
    torch.cuda.synchronize()
    assert flags.cpu().tolist()[0] == 1
    say("noalloc moving flow: latches cleared by the call")
    W = torch.tensor(I.random_smooth_state(m, seed=2, amp=0.1), device=dev)
    rd.rd_adjoint_step_noalloc(g.h, W, 1e-3, rd.B, rd.RK2, lam, out, flags)
    torch.cuda.synchronize()
    assert flags.cpu().tolist() == [0, 0]
    with pytest.raises(rd.RDError) as e:
        rd.rd_adjoint_step_noalloc(g.h, W, 1e-3, rd.BX, rd.RK2, lam, out, flags)
    assert e.value.status == rd.RD_EUNSUPPORTED
    with pytest.raises(rd.RDError) as e:
        rd.rd_adjoint_step_noalloc(g.h, W, -1.0, rd.B, rd.RK2, lam, out, flags)
    assert e.value.status == rd.RD_EINVAL
    g.close()
    say("noalloc mesh beyond the workspace")
    big = I.split_square(400)
    gb = rd.Mesh(big)
    Wb = torch.tensor(I.ic_fourier_density(big, seed=0), device=dev)
    lb = torch.zeros_like(Wb)
    with pytest.raises(rd.RDError) as e:
        rd.rd_adjoint_step_noalloc(gb.h, Wb, 1e-4, rd.B, rd.RK2, lb, torch.empty_like(lb), flags)
    assert e.value.status == rd.RD_EINVAL
    assert "workspace" in rd.rd_last_error()
    gb.close()
