"""Differentiable wrappers of the library step (torch.autograd.Function).

Every derivative is computed by the library's tangent/adjoint kernels
(cmhd_rk3_step_vjp, cmhd_bz_plane_vjp); these classes only sequence calls:

* Rk3Step: one step y = Step(x, u*) at fixed t, dt.
* rollout: n steps with checkpoints every `ckpt_every` steps; the backward
  pass recomputes each window from its checkpoint and runs the step adjoints
  in reverse (memory: n/ckpt_every states plus one window).
* bz_plane: B_z on a horizontal plane (the magnetogram-fit loss).
"""
from __future__ import annotations

import torch


class Rk3Step(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state, uh, solver, t, dt):
        solver.set_driver(uh)
        out = state.detach().clone()
        solver.rk3_step(out, t, dt)
        ctx.save_for_backward(state.detach().clone(), uh.detach())
        ctx.solver, ctx.t, ctx.dt = solver, t, dt
        return out

    @staticmethod
    def backward(ctx, ybar):
        x, uh = ctx.saved_tensors
        s = ctx.solver
        s.set_driver(uh)
        uhbar = torch.zeros_like(uh)
        xbar = s.rk3_step_vjp(x.clone(), ctx.t, ctx.dt, ybar.contiguous(), uhbar)
        return xbar, uhbar, None, None, None


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state, uh, solver, t0, dt, nsteps, ckpt_every):
        solver.set_driver(uh)
        x = state.detach().clone()
        t = t0
        ckpts = []
        for n in range(nsteps):
            if n % ckpt_every == 0:
                ckpts.append((n, x.clone(), t))
            t, _ = solver.rk3_step(x, t, dt)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.every = solver, dt, nsteps, ckpt_every
        ctx.ckpts = ckpts
        ctx.save_for_backward(uh.detach())
        return x

    @staticmethod
    def backward(ctx, ybar):
        (uh,) = ctx.saved_tensors
        s, dt = ctx.solver, ctx.dt
        s.set_driver(uh)
        uhbar = torch.zeros_like(uh)
        lam = ybar.contiguous()
        for n0, xc, tc in reversed(ctx.ckpts):
            nw = min(ctx.every, ctx.nsteps - n0)
            states, times = [xc.clone()], [tc]
            for _ in range(nw - 1):
                x = states[-1].clone()
                t, _ = s.rk3_step(x, times[-1], dt)
                states.append(x)
                times.append(t)
            for i in reversed(range(nw)):
                lam = s.rk3_step_vjp(states[i].clone(), times[i], dt, lam, uhbar)
        return lam, uhbar, None, None, None, None, None


def rollout(solver, state, uh, t0, dt, nsteps, ckpt_every=5):
    """State after nsteps steps from t0, differentiable in state and u*."""
    return _Rollout.apply(state, uh, solver, t0, dt, nsteps, ckpt_every)


class _BzPlane(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state, solver, z):
        ctx.solver, ctx.z = solver, z
        ctx.shape = state.shape
        return solver.bz_plane(state.detach(), z)

    @staticmethod
    def backward(ctx, bzbar):
        xbar = torch.zeros(ctx.shape, dtype=torch.float64, device=bzbar.device)
        ctx.solver.bz_plane_vjp(ctx.z, bzbar.contiguous(), xbar)
        return xbar, None, None


def bz_plane(solver, state, z):
    return _BzPlane.apply(state, solver, z)


def bz_misfit_loss(solver, state, z, target):
    """L = 1/2 sum_xy (B_z(x, y, z) - target)^2."""
    d = bz_plane(solver, state, z) - target
    return 0.5 * (d * d).sum()
