"""Differentiable rollout of the HDM lattice Boltzmann step on the GPU.

``HDMRollout.apply(rho0, g, T, params, nsteps, every)`` returns the density
after ``nsteps`` steps from f = f^eq(rho0, 0).  Its backward pass is the
library's hand-written adjoint step (lbm_adjoint_step) driven in reverse with
sqrt(N)-style checkpointing: the forward pass keeps one state snapshot every
``every`` steps; the backward pass reloads each snapshot, recomputes its
segment into ``every + 1`` slots (lbm_record) and runs its adjoint steps in
reverse order in one call (lbm_adjoint_steps).  Memory: ceil(nsteps / every)
+ every + 1 snapshots.  Gradients flow to
rho0, to the interaction multiplier g and to the temperature T.
"""
import dataclasses
import math

import torch

from . import Domain, Params


def _check_schedule(nsteps: int, every: int):
    if int(nsteps) != nsteps or nsteps < 0:
        raise ValueError(f"nsteps must be a non-negative integer (got {nsteps})")
    if int(every) != every or every < 1:
        raise ValueError(f"every (steps between snapshots) must be a positive integer (got {every})")


class HDMRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, g, T, params: Params, nsteps: int, every: int = 70):
        _check_schedule(nsteps, every)
        p = dataclasses.replace(params, g=float(g), T=float(T), prec="f64")
        d = Domain(p, rho0.detach().contiguous())
        nseg = max(1, math.ceil(nsteps / every))
        ck = d.new_states(nseg)
        for sidx in range(nseg):
            d.save_state(ck[sidx])
            d.step(min(every, nsteps - sidx * every))
        rho = d.moments(want=("rho",))["rho"]
        ctx.d, ctx.ck, ctx.nsteps, ctx.every = d, ck, nsteps, every
        ctx.g_dev, ctx.T_dev = g, T
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        d, ck, nsteps, every = ctx.d, ctx.ck, ctx.nsteps, ctx.every
        ny, nx = grad_rho.shape
        # rho = sum_i f_i, so dJ/df_i = dJ/drho for every population
        lam = grad_rho.detach().to(torch.float64).expand(9, ny, nx).contiguous()
        lam2 = torch.empty_like(lam)
        grad = torch.zeros(2, dtype=torch.float64, device=lam.device)
        ws = d.adjoint_workspace()
        seg = d.new_states(min(every, max(nsteps, 1)) + 1)
        nseg = max(1, math.ceil(nsteps / every))
        for sidx in reversed(range(nseg)):
            t0, t1 = sidx * every, min(nsteps, sidx * every + every)
            if t1 <= t0:
                continue
            d.load_state(ck[sidx])
            d.record(seg, t1 - t0)
            d.adjoint_steps(seg, t1 - t0, lam, lam2, grad, ws)
        drho0 = d.adjoint_rho0(lam)

        def like(v, ref):
            return v.to(dtype=ref.dtype, device=ref.device).reshape(ref.shape) if torch.is_tensor(ref) else None

        return drho0, like(grad[0], ctx.g_dev), like(grad[1], ctx.T_dev), None, None, None


def rollout(rho0, g, T, params: Params, nsteps: int, every: int = 70):
    """Density after nsteps steps, differentiable in rho0, g and T."""
    return HDMRollout.apply(rho0, g, T, params, nsteps, every)
