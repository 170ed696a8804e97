"""Differentiable wall-stress / flow-rate loss of a lattice Boltzmann run (torch autograd).

The loss L(theta) = lw0 <(W_bot + W_top)/2> + lw1 <Q> over T steps from a fixed initial state
(emulsion section: wall stress and flow rate of a confined, pressure-driven emulsion) is a
function of theta = (G_AA,1, G_BB,1, G_AA,2, G_BB,2, G_AB, g_x).  Its value and gradient
come from one call of the library's hand-written adjoint (lb_adjoint), wrapped in a
torch.autograd.Function so that theta can be produced by any differentiable torch
expression (e.g. one G1 shared by both species).
"""

import numpy as np
import torch

__all__ = ["ChannelLoss", "channel_loss"]


class ChannelLoss(torch.autograd.Function):
    """forward(theta, sim, f0, T, loss_weights, every, fp64_reverse) -> L (float64 scalar).

    sim: a Sim whose couplings and wall densities define the problem; f0: canonical FP64
    populations (device tensor) of the initial state, restored before every evaluation.
    fp64_reverse: run the reverse sweep in FP64 over the states recomputed in the storage
    precision.  The parameter sensitivities are sums over the lattice of terms that cancel
    (pair forces sum to zero), so FP32 reverse arithmetic loses about three digits over long
    horizons; the FP64 reverse sweep keeps the gradient of an FP32 forward within ~1e-6.
    Gradients flow to theta only."""

    @staticmethod
    def forward(ctx, theta, sim, f0, T, loss_weights, every, fp64_reverse):
        th = [float(v) for v in theta.detach().cpu().numpy()]
        sim.restore(f0)
        sim.set_couplings(g1=(th[0], th[1]), g2=(th[2], th[3]), gab=th[4], body=(th[5], sim._ckw["body"][1]))
        loss, grad = sim.adjoint(T, loss_weights, every, fp64_reverse=fp64_reverse)
        ctx.save_for_backward(torch.tensor(grad[:6], dtype=theta.dtype, device=theta.device))
        return torch.tensor(loss, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout * g, None, None, None, None, None, None


def channel_loss(theta, sim, f0, T, loss_weights=(1.0, 0.0), every=0, fp64_reverse=True):
    return ChannelLoss.apply(theta, sim, f0, int(T), tuple(float(v) for v in loss_weights), int(every),
                             bool(fp64_reverse))
