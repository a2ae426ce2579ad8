"""torch.autograd wrappers of the tracer step and its hand-written adjoint.

``TracerSteps.apply(T0, kappa, model, n_steps, checkpoint_every)`` advances
``T0`` by ``n_steps`` library steps and returns the final state.  Its backward
runs the library's adjoint step in reverse: the forward pass keeps only every
``checkpoint_every``-th state (and the states of the last segment, which is
reversed first); each earlier segment is recomputed from its checkpoint
(storing the states it needs) and then reversed step by step.  The adjoint
state is carried as Z = M^-1 lambda; the returned gradients are
dJ/dT0 = M Z_0 and dJ/dkappa (per layer).  Both time schemes are reversed:
SSP-RK3 + Lie with the state after each step, split-IMEX with each step's
vertically implicit half-step state x_h (kept by ``step_keep_half``, so the
reverse step need not rebuild it).

``MNorm.apply(x, model)`` is J = sqrt(sum_f x_f^T M x_f), whose gradient is
M x / J.  Both use only library kernels on the device.
"""

from __future__ import annotations

import math

import torch

from .slimdg import SDG_SCHEME_SPLIT_IMEX, SDG_SCHEME_SSPRK3_LIE


def _imex(model) -> bool:
    return getattr(model, "time_scheme", SDG_SCHEME_SSPRK3_LIE) == SDG_SCHEME_SPLIT_IMEX


def _segment_states(model, state, k):
    """k steps of `model` on its set fields `state`, keeping what their
    reversal needs: SSP-RK3 + Lie, the states before step 0 .. after step
    k-1 (k + 1 of them); split-IMEX, each step's half-step state x_h (k)."""
    if _imex(model):
        xs = []
        for _ in range(k):
            xh = torch.empty_like(state)
            model.step_keep_half(xh)
            xs.append(xh)
        return xs
    xs = [state.clone()]
    for _ in range(k):
        model.step(1)
        xs.append(state.clone())
    return xs


class TracerSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T0, kappa, model, n_steps: int, checkpoint_every: int = 20):
        if model.dtype != torch.float64:
            raise ValueError("the adjoint needs an FP64 model")
        kap = kappa.detach().contiguous()
        model.set_diffusivity(kap)
        state = T0.detach().clone()
        model.set_fields(state)
        ckpts = []
        last = None
        done = 0
        while done < n_steps:
            ckpts.append(state.clone())
            k = min(checkpoint_every, n_steps - done)
            if done + k == n_steps:
                # the last segment's states are kept as they are computed: its
                # reversal starts right away and needs no recomputation
                last = _segment_states(model, state, k)
            else:
                model.step(k)
            done += k
        ctx.model = model
        ctx.ckpts = ckpts
        ctx.last = last
        ctx.n_steps = n_steps
        ctx.every = checkpoint_every
        ctx.kappa = kap
        return state

    @staticmethod
    def backward(ctx, grad_xN):
        s = ctx.model
        s.set_diffusivity(ctx.kappa)
        z = s.apply_mass(grad_xN.contiguous(), inverse=True)
        dk = torch.zeros_like(ctx.kappa)
        for i in range(len(ctx.ckpts) - 1, -1, -1):
            start = i * ctx.every
            k = min(ctx.every, ctx.n_steps - start)
            if i == len(ctx.ckpts) - 1 and ctx.last is not None:
                xs = ctx.last                    # kept by the forward pass
                ctx.last = None
            else:
                st = ctx.ckpts[i].clone()
                s.set_fields(st)
                xs = _segment_states(s, st, k)
            for j in range(k - 1, -1, -1):
                if _imex(s):
                    # the split-IMEX reverse step takes that step's x_h
                    zn = torch.empty_like(z)
                    s.step_adjoint_imex_half(z, zn, xs[j], dk)
                    z = zn
                else:
                    s.step_adjoint(z, z, xs[j + 1], dk)
        grad_T0 = s.apply_mass(z)
        return grad_T0, dk, None, None, None


class MNorm(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, model):
        v = float(model.m_dot(x, x).sum())
        J = math.sqrt(v)
        ctx.model = model
        ctx.save_for_backward(x)
        ctx.J = J
        return torch.tensor(J, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, gJ):
        (x,) = ctx.saved_tensors
        g = ctx.model.apply_mass(x.contiguous())
        return g * (gJ / ctx.J), None
