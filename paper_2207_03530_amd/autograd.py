"""torch.autograd wrappers of the HIP step and rollout.

Forward passes call vmas_step / vmas_rollout, backward passes the
hand-written adjoint (vmas_step_backward / vmas_rollout_backward, which
replays the rollout from checkpoints stored every `ckpt_every` steps).
Gradients flow to the initial state and to the actions; the static batch
description is not differentiated.
"""
from __future__ import annotations

import torch

from .binding import Batch


class VmasStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state, actions, batch: Batch):
        out = state.detach().clone().contiguous()
        batch.step(out, actions.detach().contiguous())
        ctx.save_for_backward(state.detach().contiguous(), actions.detach().contiguous())
        ctx.batch = batch
        return out

    @staticmethod
    def backward(ctx, grad_out):
        state, actions = ctx.saved_tensors
        gs = torch.empty_like(state)
        ga = torch.empty_like(actions)
        ctx.batch.step_backward(state, actions, grad_out.contiguous(), gs, ga)
        return gs, ga, None


class VmasRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, state0, actions, batch: Batch, ckpt_every: int):
        out = state0.detach().clone().contiguous()
        batch.rollout(out, actions.detach().contiguous())
        ctx.save_for_backward(state0.detach().contiguous(), actions.detach().contiguous())
        ctx.batch = batch
        ctx.ckpt_every = int(ckpt_every)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        state0, actions = ctx.saved_tensors
        gs = torch.empty_like(state0)
        ga = torch.empty_like(actions)
        ctx.batch.rollout_backward(state0, actions, grad_out.contiguous(), ctx.ckpt_every, gs, ga)
        return gs, ga, None, None


def step(batch: Batch, state, actions):
    """Differentiable single step: state [6, N], actions [A, 2] -> state [6, N]."""
    return VmasStep.apply(state, actions, batch)


def rollout(batch: Batch, state0, actions, ckpt_every: int = 10):
    """Differentiable T-step rollout: state0 [6, N], actions [T, A, 2] -> final state."""
    return VmasRollout.apply(state0, actions, batch, ckpt_every)
