"""Joule loss of the semi-explicit time loop as a torch.autograd.Function.

forward runs the time loop on the GPU with checkpoints (ec_adjoint_forward);
backward recomputes segments from them and runs the hand-written discrete
adjoint (ec_adjoint_backward).  Gradients are with respect to the
conductivity sigma and the Brauer coefficient k1 (eq. 1) of one material.
"""
from __future__ import annotations

import torch


class EddyLoss(torch.autograd.Function):
    """loss = EddyLoss.apply(sigma, k1, problem, dt, n_steps, every, opts, mat_id)

    sigma and k1 are 0-d float64 tensors (any device); problem is a
    paper_1611_06721_amd.Problem whose material mat_id (with its k2, k3) is
    replaced by (sigma, k1) before the run; opts are step options (start
    vector, tolerance) for the forward steps and the adjoint solves."""

    @staticmethod
    def forward(ctx, sigma, k1, problem, dt, n_steps, every, opts, mat_id=1):
        wl_mat = problem.wl.materials[mat_id - 1]
        problem.set_material(mat_id, float(sigma), float(k1), wl_mat.k2, wl_mat.k3)
        ws = problem.adjoint_workspace(n_steps, every)
        A = problem.zeros()
        loss = problem.adjoint_forward(A, n_steps, dt, every, opts, ws)
        ctx.problem, ctx.ws = problem, ws
        ctx.args = (n_steps, dt, every, opts, mat_id)
        ctx.dev = sigma.device
        return loss[0].to(sigma.device)

    @staticmethod
    def backward(ctx, grad_out):
        n_steps, dt, every, opts, mat_id = ctx.args
        g = ctx.problem.adjoint_backward(n_steps, dt, every, opts, ctx.ws, mat_id).to(ctx.dev)
        ctx.ws = None
        return (grad_out * g[0], grad_out * g[1], None, None, None, None, None, None)


def eddy_loss(sigma, k1, problem, dt, n_steps, every=50, opts=None, mat_id=1):
    from .problem import step_opts
    if opts is None:
        opts = step_opts()
    return EddyLoss.apply(sigma, k1, problem, dt, n_steps, every, opts, mat_id)
