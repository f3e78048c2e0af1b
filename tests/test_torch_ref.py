"""Pins of the torch-CPU reference gradient (oracle/torch_ref.py).

Its eigenvectors are checked against the mathematics (R^{-1} R = I, K equal
to a finite-difference Jacobian of the Euler flux along the normal, K^+ with
eigenvalues max(lambda, 0)); its step against the C++ oracle (which has its
own pins); its reverse-mode derivative against the oracle's forward-mode
(dual number) derivative, and against central differences where the scheme
is smooth (LDA)."""
import numpy as np
import pytest
import torch

import oracle as orc
import torch_ref as tr
from paper_1705_02028_amd import inputs as I


def euler_flux_n(W, nx, ny, gamma):
    """F(W).n for the 2D Euler equations written from their definition."""
    rho, mx, my, e = W
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (e - 0.5 * rho * (u * u + v * v))
    un = u * nx + v * ny
    return np.array([rho * un, mx * un + p * nx, my * un + p * ny, (e + p) * un])


def _state(rng, gamma=1.4):
    rho = rng.uniform(0.3, 2.0)
    u, v = rng.uniform(-1.5, 1.5, size=2)
    p = rng.uniform(0.2, 3.0)
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def _roe_quantities(W, gamma=1.4):
    rho = W[0]
    u, v = W[1] / rho, W[2] / rho
    p = (gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v))
    h = (W[3] + p) / rho
    c = np.sqrt(gamma * p / rho)
    return u, v, h, c


def test_left_eigenvectors_invert_right_ones():
    rng = np.random.default_rng(0)
    for _ in range(50):
        u, v, h, c = _roe_quantities(_state(rng))
        th = rng.uniform(0, 2 * np.pi)
        _, _, _, R, L = tr.eigen_split(*(torch.tensor(q) for q in (u, v, h, c, np.cos(th), np.sin(th))), 1.4)
        assert np.abs((L @ R).numpy() - np.eye(4)).max() < 1e-13
        assert np.abs((R @ L).numpy() - np.eye(4)).max() < 1e-13


def test_split_matches_flux_jacobian_and_eigenvalues():
    """K = dF.n/dW by central differences of the flux; K^+ has eigenvalues
    max(lambda, 0) and K^- min(lambda, 0) with lambda = (w + c, w - c, w, w)."""
    rng = np.random.default_rng(1)
    g = 1.4
    for _ in range(30):
        W = _state(rng)
        u, v, h, c = _roe_quantities(W)
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        K, Kp, Km, _, _ = (t.numpy() for t in tr.eigen_split(
            *(torch.tensor(q) for q in (u, v, h, c, nx, ny)), g))
        J = np.zeros((4, 4))
        for j in range(4):
            e = np.zeros(4)
            e[j] = 1e-6 * max(1.0, abs(W[j]))
            J[:, j] = (euler_flux_n(W + e, nx, ny, g) - euler_flux_n(W - e, nx, ny, g)) / (2 * e[j])
        assert np.abs(K - J).max() <= 1e-7 * np.abs(J).max()
        assert np.abs(Kp + Km - K).max() <= 1e-13 * np.abs(K).max()
        w = u * nx + v * ny
        lam = np.sort([w + c, w - c, w, w])
        assert np.allclose(np.sort(np.linalg.eigvals(Kp).real), np.sort(np.maximum(lam, 0)), atol=1e-12)
        assert np.allclose(np.sort(np.linalg.eigvals(Km).real), np.sort(np.minimum(lam, 0)), atol=1e-12)


MESHES = {
    "periodic_random": lambda: I.split_square(17, diagonal="random", jitter=0.15, seed=1),
    "ghost_walls": lambda: I.split_square(15, periodic=(False, False), bc=("ghost", "wall"),
                                          diagonal="random", seed=2),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_step_and_vjp_match_the_oracle(name):
    """Forward step equal to the C++ oracle's to rounding; <lam, J v> from the
    oracle's dual numbers equals <J^T lam, v> from torch.autograd."""
    m = MESHES[name]()
    W = I.random_smooth_state(m, seed=3, amp=0.2)
    om = orc.OracleMesh(m)
    tm = tr.TorchMesh(m)
    dt = om.max_dt(W, 0.4)
    rng = np.random.default_rng(4)
    for scheme in (tr.N, tr.LDA, tr.B, tr.BMAX, tr.BMIN):
        for time_order in (tr.EULER1, tr.RK2):
            ref = om.step(W, dt, scheme, time_order)
            Wt = torch.tensor(W, requires_grad=True)
            out = tr.step(tm, Wt, dt, scheme, time_order)
            got = out.detach().numpy()
            for k in range(4):
                assert np.abs(got[k] - ref[k]).max() <= 1e-14 * np.abs(ref[k]).max()
            v = rng.normal(size=W.shape) * np.abs(W).mean(axis=1, keepdims=True)
            lam = rng.normal(size=W.shape)
            (out * torch.tensor(lam)).sum().backward()
            _, Jv = om.step_jvp(W, v, dt, scheme, time_order)
            a, b = float(np.sum(lam * Jv)), float(np.sum(Wt.grad.numpy() * v))
            assert abs(a - b) <= 1e-13 * float(np.sum(np.abs(lam * Jv)))


def test_rollout_gradient_against_dual_rollout_and_differences():
    """The density gradient of the rollout loss: every component against the
    oracle's forward-mode rollout on single-vertex directions (a sample of
    vertices), and (LDA, no kinks) against central differences."""
    m = I.split_square(13)
    W0 = I.ic_fourier_density(m, seed=0)
    target = I.ic_fourier_density(m, seed=1)[0]
    om = orc.OracleMesh(m)
    dt = om.max_dt(W0, 0.4)
    n = 12
    u, v = 0.5, 0.3
    for scheme in (tr.B, tr.LDA):
        L, grad, _ = tr.rollout_density_gradient(m, W0[0], target, dt, n, scheme)
        for i in (0, 7, 50, m["nv"] - 1):
            d = np.zeros(m["nv"])
            d[i] = 1.0
            Wd = np.stack([d, d * u, d * v, 0.5 * d * (u * u + v * v)])
            Wc = W0.copy()
            for _ in range(n):
                Wc, Wd = om.step_jvp(Wc, Wd, dt, scheme, orc.RK2)
            exact = float(np.sum(2.0 * (Wc[0] - target) * Wd[0]))
            assert abs(grad[i] - exact) <= 1e-12 * np.abs(grad).max()
        if scheme == tr.LDA:
            d = np.random.default_rng(2).normal(size=m["nv"])
            eps = 1e-6
            Lp = tr.rollout_density_gradient(m, W0[0] + eps * d, target, dt, n, scheme)[0]
            Lm = tr.rollout_density_gradient(m, W0[0] - eps * d, target, dt, n, scheme)[0]
            fd = (Lp - Lm) / (2 * eps)
            assert abs(fd - float(grad @ d)) <= 1e-6 * abs(fd)
