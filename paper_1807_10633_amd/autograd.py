"""The gradient-ratio backward as a torch.autograd.Function.

``vmc_energy(system, walkers, J, theta)`` returns the residence-time weighted
energy of the current walker states, E = sum_w t_w E_L,w / sum_w t_w (Eq. eq:vmc
sampled with CTMC weights).  Its backward is not the derivative of that sample
mean: it is the VMC gradient estimator of Eq. eq:grad,
G_k = 2 < O_k (E_L - E) >, computed by the library's contracted backward with
g_w = 2 t_w (E_L,w - E) / sum t and returned as gradients of J (packed) and
theta.  Local energies come from the library's kernels (vmc_local_energy), the
weighted mean and the weights g from vmc_estimate, the contraction from
vmc_logderiv; torch only holds memory.
"""
from __future__ import annotations

import torch

from . import vmc as _vmc


class _VMCEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, J, theta, system, walkers):
        if J.device.type != "cuda":
            raise RuntimeError("vmc_energy runs on the GPU only")
        _vmc.vmc_local_energy(system.handle, walkers)
        W = walkers.n_walkers
        est = torch.empty(4, dtype=torch.float64, device=J.device)
        g = torch.empty(W, dtype=torch.float64, device=J.device)
        _vmc.vmc_estimate(system.handle, walkers, est, g)
        ctx.system = system
        ctx.walkers = walkers
        ctx.save_for_backward(g)
        ctx.shapes = (J.shape, theta.shape)
        return est[2].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        system, walkers = ctx.system, ctx.walkers
        G = torch.empty(system.n_params, dtype=torch.float64, device=g.device)
        _vmc.vmc_logderiv(system.handle, walkers, g, G)
        nj = system.n_so * (system.n_so + 1) // 2
        nt = system.n_so * system.n_so
        gJ = (grad_out * G[:nj]).reshape(ctx.shapes[0])
        gT = (grad_out * G[nj:nj + nt]).reshape(ctx.shapes[1])
        return gJ, gT, None, None


def vmc_energy(system, walkers, J, theta):
    """Weighted VMC energy with the Eq. eq:grad estimator as its backward.

    J (packed upper triangle) and theta must be the tensors last passed to
    ``system.set_params``.
    """
    return _VMCEnergy.apply(J, theta, system, walkers)
