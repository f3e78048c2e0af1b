"""Differentiable steps on top of the C ABI.

``RDStep.apply(W, mesh, dt, scheme, time)`` is one step with its adjoint as
the backward. ``RDRollout.apply(W0, mesh, dt, n_steps, scheme, time, checkpoint_every)``
advances the state ``W0`` (a float64 tensor [4, nv] on the GPU) by
``n_steps`` steps of fixed size ``dt`` with ``rd_step`` and returns the final
state. Its backward pass uses ``rd_adjoint_step`` (the hand-written reverse
of one step): the forward keeps only every ``checkpoint_every``-th state;
the backward replays each segment forward from its checkpoint, keeping that
segment's states, and then runs the adjoint steps of the segment in reverse.
Memory is (n_steps / checkpoint_every + checkpoint_every) states; work is
about one extra forward pass. The time step is held fixed (it is not
differentiated). All arithmetic runs in librd's kernels; torch provides the
buffers and the stream.
"""
from __future__ import annotations

import torch

from . import rd


def _state(mesh, like):
    out = torch.empty_like(like)
    rd.rd_get_state(mesh.h, out)
    return out


class RDStep(torch.autograd.Function):
    """One step: ``RDStep.apply(W, mesh, dt, scheme, time)`` returns the state
    after ``rd_step`` (fixed ``dt``, FP64); its backward is ``rd_adjoint_step``
    at the saved input state."""

    @staticmethod
    def forward(ctx, W, mesh, dt, scheme=rd.B, time=rd.RK2):
        if W.dtype != torch.float64 or not W.is_cuda:
            raise ValueError("W must be a float64 tensor on the GPU")
        W = W.contiguous()
        rd.rd_set_state(mesh.h, W)
        rd.rd_step(mesh.h, dt, scheme, time, rd.FP64)
        out = _state(mesh, W)
        ctx.mesh = mesh
        ctx.args = (float(dt), int(scheme), int(time))
        ctx.save_for_backward(W)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (W,) = ctx.saved_tensors
        dt, scheme, time = ctx.args
        lam = grad_out.contiguous().to(torch.float64)
        out = torch.empty_like(lam)
        rd.rd_adjoint_step(ctx.mesh.h, W, dt, scheme, time, lam, out)
        rd.rd_sync(ctx.mesh.h)  # raises on a latched non-physical or singular (stagnant) case
        return out, None, None, None, None


class RDRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W0, mesh, dt, n_steps, scheme=rd.B, time=rd.RK2, checkpoint_every=20):
        if W0.dtype != torch.float64 or not W0.is_cuda:
            raise ValueError("W0 must be a float64 tensor on the GPU")
        W0 = W0.contiguous()
        k = max(1, int(checkpoint_every))
        ckpts = []
        rd.rd_set_state(mesh.h, W0)
        for s in range(n_steps):
            if s % k == 0:
                ckpts.append(_state(mesh, W0))
            rd.rd_step(mesh.h, dt, scheme, time, rd.FP64)
        out = _state(mesh, W0)
        ctx.mesh = mesh
        ctx.args = (float(dt), int(n_steps), int(scheme), int(time), k)
        ctx.ckpts = ckpts
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mesh = ctx.mesh
        dt, n_steps, scheme, time, k = ctx.args
        lam = grad_out.contiguous().to(torch.float64)
        nxt = torch.empty_like(lam)
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * k
            s1 = min(n_steps, s0 + k)
            states = [ctx.ckpts[seg]]
            rd.rd_set_state(mesh.h, states[0])
            for _ in range(s0, s1 - 1):
                rd.rd_step(mesh.h, dt, scheme, time, rd.FP64)
                states.append(_state(mesh, lam))
            for s in reversed(range(s0, s1)):
                rd.rd_adjoint_step(mesh.h, states[s - s0], dt, scheme, time, lam, nxt)
                lam, nxt = nxt, lam
        ctx.ckpts = None
        rd.rd_sync(mesh.h)  # raises on a latched non-physical or singular (stagnant) case
        return lam, None, None, None, None, None, None


def conserved_from_density(rho, u, v, p, gamma):
    """W = (rho, rho u, rho v, rho (u^2 + v^2)/2 + p/(gamma - 1)) in torch, so
    gradients flow from W back to the density at fixed velocity and pressure."""
    rho_u = rho * u
    rho_v = rho * v
    e = 0.5 * rho * (u * u + v * v) + p / (gamma - 1.0)
    return torch.stack([rho, rho_u, rho_v, e])
