"""Vectorised torch-CPU FP64 form of the residual-distribution step, for
reference gradients by reverse-mode automatic differentiation.

TEST INFRASTRUCTURE ONLY: imported by the tests and nothing else; it never
touches a GPU. It restates one step of the method (Sections 3.2-3.5) over
whole arrays of triangles so that ``torch.autograd`` gives the exact gradient
of a multi-step loss, as a second reference beside the C++ oracle's
forward-mode (dual number) derivative.

It is written independently of both the C++ oracle and the GPU library:
 * K_i^{+-} come from the eigen-decomposition K = R diag(lambda) R^{-1} of the
   flux Jacobian along the unit normal, with right and left eigenvectors
   written out in closed form (the decomposition Appendix A starts from; its
   printed inverse carries a sign error in the fourth column, so the left
   eigenvectors here are derived directly and checked by R^{-1} R = I in the
   tests), not from Appendix A's explicit entries;
 * the two 4x4 systems per triangle are solved by ``torch.linalg.solve``
   (LAPACK's LU with partial pivoting); no stagnant triangle is supported
   (A is singular at rest: the pivot-skip rule is not reproduced);
 * vertex sums use ``index_add`` (summation order is immaterial at the
   tolerances this serves).

Derivative conventions (Section 3.3 branches): d max(x, 0)/dx = [x > 0],
d min(x, 0)/dx = [x < 0], d|x|/dx = sign(x) with sign(0) = 0, zero derivative
in the 0/0 branch of the blend coefficient and where it is clamped to 1.
Readings of the paper follow the C++ oracle's header: Z = sqrt(rho)(1, u, v, h);
K_i = (|n_i| / 2) K(n_i / |n_i|) with n_i the inward normal scaled by the
edge length; state differences M(Zbar)(Z_i - Z_0); median-dual vertex
volumes; stage 2 of the Runge-Kutta scheme with global lumping, the LDA
coefficients at W*, and the wall term averaged over both stages.
"""
from __future__ import annotations

import numpy as np
import torch

N, LDA, B, BMAX, BMIN = 0, 1, 2, 3, 4
EULER1, RK2 = 1, 2
DT = torch.float64


def _unwrap(d, period):
    if period > 0.0:
        d = np.where(d > 0.5 * period, d - period, d)
        d = np.where(d < -0.5 * period, d + period, d)
    return d


class TorchMesh:
    """Geometry of a mesh dict (``paper_1705_02028_amd.inputs``) as tensors
    (Section 3.2): areas, inward scaled normals, median-dual volumes, wall
    edges with their outward unit normals (Section 3.5)."""

    def __init__(self, mesh: dict):
        self.nv = int(mesh["nv"])
        self.nt = int(mesh["nt"])
        self.gamma = float(mesh.get("gamma", 1.4))
        x = np.asarray(mesh["x"], np.float64)
        y = np.asarray(mesh["y"], np.float64)
        tri = np.asarray(mesh["tri"], np.int64).reshape(-1, 3)
        px, py = float(mesh["px"]), float(mesh["py"])
        # corner positions relative to corner 0 on the minimum image
        rel = np.zeros((self.nt, 3, 2))
        for k in (1, 2):
            rel[:, k, 0] = _unwrap(x[tri[:, k]] - x[tri[:, 0]], px)
            rel[:, k, 1] = _unwrap(y[tri[:, k]] - y[tri[:, 0]], py)
        e1, e2 = rel[:, 1], rel[:, 2]
        area = 0.5 * (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        if not np.all(area > 0.0):
            raise ValueError("triangles must be counter-clockwise with positive area")
        # edge opposite corner i runs from corner i+1 to corner i+2; the inward
        # normal is that edge turned a quarter turn counter-clockwise
        edge = np.stack([rel[:, 2] - rel[:, 1], rel[:, 0] - rel[:, 2], rel[:, 1] - rel[:, 0]], axis=1)
        nrm = np.stack([-edge[..., 1], edge[..., 0]], axis=-1)
        length = np.sqrt((nrm ** 2).sum(-1))
        V = np.zeros(self.nv)
        np.add.at(V, tri.reshape(-1), np.repeat(area / 3.0, 3))
        self.tri = torch.as_tensor(tri)
        self.area = torch.as_tensor(area, dtype=DT)
        self.len = torch.as_tensor(length, dtype=DT)               # [nt, 3]
        self.nhat = torch.as_tensor(nrm / length[..., None], dtype=DT)  # [nt, 3, 2]
        self.V = torch.as_tensor(V, dtype=DT)
        self.ghost = torch.as_tensor(np.asarray(mesh["ghost"]).astype(bool))
        wall = np.asarray(mesh["wall"], np.int64).reshape(-1, 2)
        self.wall = torch.as_tensor(wall)
        if wall.size:
            dx = _unwrap(x[wall[:, 1]] - x[wall[:, 0]], px)
            dy = _unwrap(y[wall[:, 1]] - y[wall[:, 0]], py)
            wl = np.sqrt(dx * dx + dy * dy)
            # the domain lies to the left of a -> b: outward is the right-hand normal
            self.wlen = torch.as_tensor(wl, dtype=DT)
            self.wn = torch.as_tensor(np.stack([dy / wl, -dx / wl], axis=1), dtype=DT)


def primitives(W, gamma):
    """(rho, u, v, p, h) of a conserved state W [4, ...]."""
    rho = W[0]
    u = W[1] / rho
    v = W[2] / rho
    p = (gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v))
    h = (W[3] + p) / rho
    return rho, u, v, p, h


def parameter_vector(W, gamma):
    """Z = sqrt(rho) (1, u, v, h) [4, nv] (Section 3.2)."""
    rho, u, v, _, h = primitives(W, gamma)
    s = torch.sqrt(rho)
    return torch.stack([s, s * u, s * v, s * h])


def eigen_split(u, v, h, c, nx, ny, gamma):
    """K, K^+ and K^- of the flux Jacobian dF.n/dW along the unit normal
    (nx, ny) at the state (u, v, h, c), as R diag(l) L with the right
    eigenvectors R (columns: acoustic w + c, acoustic w - c, entropy w,
    shear w) and left eigenvectors L = R^{-1}. Shapes broadcast; the matrix
    dimensions are last: [..., 4, 4]."""
    g1 = gamma - 1.0
    u, v, h, c, nx, ny = torch.broadcast_tensors(u, v, h, c, nx, ny)
    w = u * nx + v * ny
    q2 = u * u + v * v
    one = torch.ones_like(w)
    zero = torch.zeros_like(w)
    R = torch.stack([
        torch.stack([one, one, one, zero], -1),
        torch.stack([u + c * nx, u - c * nx, u, -ny * one], -1),
        torch.stack([v + c * ny, v - c * ny, v, nx * one], -1),
        torch.stack([h + c * w, h - c * w, 0.5 * q2, v * nx - u * ny], -1),
    ], -2)
    a = 0.5 * g1 * q2
    c2 = c * c
    L = torch.stack([
        torch.stack([(a - c * w) / (2 * c2), (c * nx - g1 * u) / (2 * c2), (c * ny - g1 * v) / (2 * c2),
                     g1 / (2 * c2) * one], -1),
        torch.stack([(a + c * w) / (2 * c2), (-c * nx - g1 * u) / (2 * c2), (-c * ny - g1 * v) / (2 * c2),
                     g1 / (2 * c2) * one], -1),
        torch.stack([1.0 - a / c2, g1 * u / c2, g1 * v / c2, -g1 / c2 * one], -1),
        torch.stack([u * ny - v * nx, -ny * one, nx * one, zero], -1),
    ], -2)
    lam = torch.stack([w + c, w - c, w, w], -1)
    lp = torch.relu(lam)        # derivative [l > 0]
    lm = -torch.relu(-lam)      # derivative [l < 0]
    K = R @ (lam[..., :, None] * L)
    Kp = R @ (lp[..., :, None] * L)
    Km = R @ (lm[..., :, None] * L)
    return K, Kp, Km, R, L


def triangles(tm: TorchMesh, Z):
    """Per-triangle quantities of Sections 3.2-3.3 at the parameter vectors Z
    [4, nv]: the state differences dW [nt, 3, 4], K_i^+ [nt, 3, 4, 4],
    A = sum K_i^+ [nt, 4, 4], phi^T [nt, 4] and the N parts [nt, 3, 4]."""
    g = tm.gamma
    g1 = g - 1.0
    Zc = Z[:, tm.tri]                         # [4, nt, 3]
    zb = Zc.sum(-1) / 3.0                     # Roe average, [4, nt]
    u, v, h = zb[1] / zb[0], zb[2] / zb[0], zb[3] / zb[0]
    c = torch.sqrt(g1 * (h - 0.5 * (u * u + v * v)))
    dz = Zc - Zc[:, :, :1]                    # Z_i - Z_0
    # M(Zbar) = dW/dZ at the Roe average applied to the differences
    dW = torch.stack([
        2.0 * zb[0, :, None] * dz[0],
        zb[1, :, None] * dz[0] + zb[0, :, None] * dz[1],
        zb[2, :, None] * dz[0] + zb[0, :, None] * dz[2],
        (zb[3, :, None] * dz[0] + g1 * zb[1, :, None] * dz[1] + g1 * zb[2, :, None] * dz[2]
         + zb[0, :, None] * dz[3]) / g,
    ], -1)                                    # [nt, 3, 4]
    nx, ny = tm.nhat[..., 0], tm.nhat[..., 1]    # [nt, 3]
    K, Kp, Km, _, _ = eigen_split(u[:, None], v[:, None], h[:, None], c[:, None], nx, ny, g)
    half = (tm.len / 2.0)[..., None, None]
    K, Kp, Km = half * K, half * Kp, half * Km
    phiT = (K[:, 1:] @ dW[:, 1:, :, None]).squeeze(-1).sum(1)       # [nt, 4]
    A = Kp.sum(1)
    bN = (Km[:, 1:] @ dW[:, 1:, :, None]).squeeze(-1).sum(1)
    xN = torch.linalg.solve(A, bN)
    phiN = (Kp @ (dW + xN[:, None, :])[..., None]).squeeze(-1)     # [nt, 3, 4]
    return dict(dW=dW, Kp=Kp, A=A, phiT=phiT, phiN=phiN)


def blend(scheme, res, PN, PL):
    """Section 3.3: the parts of a scheme from the residual res [nt, 4], its N
    parts PN and LDA parts PL [nt, 3, 4]."""
    if scheme == N:
        return PN
    if scheme == LDA:
        return PL
    den = PN.abs().sum(1)                     # [nt, 4]
    safe = torch.where(den == 0.0, torch.ones_like(den), den)
    q = res.abs() / safe
    theta = torch.where(den == 0.0, torch.zeros_like(q), torch.where(q > 1.0, torch.ones_like(q), q))
    if scheme in (BMAX, BMIN):
        idx = (theta if scheme == BMAX else -theta).argmax(1, keepdim=True)
        theta = theta.gather(1, idx).expand(-1, 4)
    return PL + theta[:, None, :] * (PN - PL)


def gather(tm: TorchMesh, parts):
    """R_i = sum over the triangles of vertex i of its corner parts, [4, nv]."""
    R = torch.zeros(tm.nv, 4, dtype=parts.dtype)
    R = R.index_add(0, tm.tri.reshape(-1), parts.reshape(-1, 4))
    return R.T


def wall_term(tm: TorchMesh, W):
    """Section 3.5: the correction residual of the reflecting walls, [4, nv]."""
    out = torch.zeros(tm.nv, 4, dtype=W.dtype)
    if tm.wall.numel() == 0:
        return out.T
    alpha = 0.75
    a, b = tm.wall[:, 0], tm.wall[:, 1]
    _, u, v, p, _ = primitives(W, tm.gamma)

    def flux(i):
        vn = u[i] * tm.wn[:, 0] + v[i] * tm.wn[:, 1]
        return torch.stack([-vn * W[0, i], -vn * W[1, i], -vn * W[2, i], -vn * (W[3, i] + p[i])], 1)
    Fa, Fb = flux(a), flux(b)
    hl = (tm.wlen / 2.0)[:, None]
    out = out.index_add(0, a, hl * (alpha * Fa + (1.0 - alpha) * Fb))
    out = out.index_add(0, b, hl * ((1.0 - alpha) * Fa + alpha * Fb))
    return out.T


def step(tm: TorchMesh, W, dt: float, scheme=B, time_order=RK2):
    """One step (Section 3.2 forward Euler, or the two-stage scheme of
    Section 3.4) of the state W [4, nv]; differentiable in W."""
    keep = ~tm.ghost
    Z = parameter_vector(W, tm.gamma)
    s1 = triangles(tm, Z)
    xL = torch.linalg.solve(s1["A"], s1["phiT"])
    PL = (s1["Kp"] @ xL[:, None, :, None]).squeeze(-1)
    parts = blend(scheme, s1["phiT"], s1["phiN"], PL)
    wall_n = wall_term(tm, W)
    R = gather(tm, parts) + wall_n
    Ws = torch.where(keep, W - (dt / tm.V) * R, W)
    if time_order == EULER1:
        return Ws
    s2 = triangles(tm, parameter_vector(Ws, tm.gamma))
    mass = (tm.area / 3.0)[:, None, None]
    rate = ((Ws - W) / dt)[:, tm.tri].permute(1, 2, 0)        # [nt, 3, 4]
    PN = mass * rate + 0.5 * (s1["phiN"] + s2["phiN"])
    PT = mass[:, 0] * rate.sum(1) + 0.5 * (s1["phiT"] + s2["phiT"])
    x = torch.linalg.solve(s2["A"], PT)
    PL2 = (s2["Kp"] @ x[:, None, :, None]).squeeze(-1)
    parts2 = blend(scheme, PT, PN, PL2)
    R2 = gather(tm, parts2) + 0.5 * (wall_n + wall_term(tm, Ws))
    return torch.where(keep, Ws - (dt / tm.V) * R2, Ws)


def conserved_from_density(rho, u, v, p, gamma):
    """W of a density field at fixed velocity (u, v) and pressure p."""
    e = 0.5 * rho * (u * u + v * v) + p / (gamma - 1.0)
    return torch.stack([rho, rho * u, rho * v, e])


def rollout_density_gradient(mesh: dict, rho0, target, dt, n_steps, scheme=B, time_order=RK2,
                             u=0.5, v=0.3, p=1.0):
    """Loss sum_i (rho_i(T) - target_i)^2 after n_steps fixed steps from
    W(rho0) at fixed (u, v, p), and its gradient with respect to rho0
    (numpy arrays). Each step is recomputed in the backward pass
    (torch.utils.checkpoint), so memory holds one state per step."""
    from torch.utils.checkpoint import checkpoint

    tm = TorchMesh(mesh)
    r = torch.tensor(np.asarray(rho0, np.float64), requires_grad=True)
    W = conserved_from_density(r, u, v, p, tm.gamma)
    for _ in range(n_steps):
        W = checkpoint(step, tm, W, dt, scheme, time_order, use_reentrant=False)
    tgt = torch.as_tensor(np.asarray(target, np.float64))
    loss = ((W[0] - tgt) ** 2).sum()
    loss.backward()
    return float(loss.detach()), r.grad.detach().numpy().copy(), W.detach().numpy()
