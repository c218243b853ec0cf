"""Differentiation of the uniform-level advance + ghost fill.

``AdvanceFill`` is a torch.autograd.Function whose forward runs ``nsteps``
coarse steps of the GPU path (graph mode)
from q0 and returns q(T); its backward is the hand-written discrete adjoint
(fc_adjoint_step: transpose of the limited step with branches frozen at the
forward state, then transpose of the ghost copy), with checkpoints every
``checkpoint_every`` steps and the states of one segment recomputed at a
time by fc_step_uniform (leaf order in, leaf order out).  checkpoint_every=1
keeps every state in HBM instead (nsteps solution copies) and recomputes
nothing; the forward then runs fc_step_uniform, bitwise the same steps.  Shapes: [nleaves][1][mx][mx] float64 on the GPU, in the leaf order the
store was created with.
"""
from __future__ import annotations

import torch


def _times(t0, dt, n):
    """Step start times exactly as the library accumulates them (t += dt)."""
    out, t = [], float(t0)
    for _ in range(n):
        out.append(t)
        t = t + float(dt)
    return out


class AdvanceFill(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q0, store, level, dt, nsteps, checkpoint_every=16, t0=0.0):
        every = max(1, int(checkpoint_every))
        times = _times(t0, dt, nsteps + 1)
        t_end, times = times[nsteps], times[:nsteps]
        if every == 1:
            # every state kept (nsteps x the solution size of HBM): the
            # leaf-order step writes each one as a tensor of its own, so
            # nothing is copied and the backward sweep recomputes nothing
            ckpts = [q0.detach().clone()]
            for k in range(nsteps):
                ckpts.append(store.step_uniform(level, times[k], dt, ckpts[-1]))
            out = ckpts.pop()
            store.set_interior(out)  # the store ends at q(T), as after the graph path
            store.time = t_end
        else:
            store.time = t0
            store.set_interior(q0.detach())
            ckpts = [q0.detach().clone()]
            k = 0
            while k < nsteps:
                m = min(every, nsteps - k)
                store.coarse_steps(dt, m, "graph")
                k += m
                if k < nsteps:
                    ckpts.append(store.interior())  # a fresh tensor
            out = store.interior()
        ctx.store, ctx.level, ctx.dt, ctx.nsteps, ctx.every = store, level, dt, nsteps, every
        ctx.times, ctx.ckpts = times, ckpts
        return out

    @staticmethod
    def backward(ctx, grad_out):
        store, level, dt, n, every = ctx.store, ctx.level, ctx.dt, ctx.nsteps, ctx.every
        lam = grad_out.detach().to(torch.float64).contiguous()
        nseg = (n + every - 1) // every
        for seg in reversed(range(nseg)):
            a, b = seg * every, min(n, (seg + 1) * every)
            # recompute the segment's step inputs q^a .. q^(b-1), leaf order
            # to leaf order (bitwise the forward's states)
            states = [ctx.ckpts[seg]]
            for k in range(a, b - 1):
                states.append(store.step_uniform(level, ctx.times[k], dt, states[-1]))
            for k in reversed(range(a, b)):
                lam = store.adjoint_step(level, ctx.times[k], dt, states[k - a], lam)
        return lam, None, None, None, None, None, None


def loss_and_grad(store, q0, q_target, level, dt, nsteps, checkpoint_every=16):
    """L = 1/2 sum (q(T) - q_target)^2 over interior cells and dL/dq0."""
    q0 = q0.detach().clone().requires_grad_(True)
    qT = AdvanceFill.apply(q0, store, level, dt, nsteps, checkpoint_every)
    L = 0.5 * ((qT - q_target) ** 2).sum()
    L.backward()
    return L.detach(), q0.grad.detach()


def loss(store, q0, q_target, dt, nsteps):
    """Forward-only loss (for finite differences)."""
    store.time = 0.0
    store.set_interior(q0)
    store.coarse_steps(dt, nsteps, "graph")
    return 0.5 * ((store.interior() - q_target) ** 2).sum()
