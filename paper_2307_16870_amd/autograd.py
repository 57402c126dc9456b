"""torch.autograd.Function around mps_energy_grad.

The forward pass runs the circuit, the energy and its reverse pass in the
library (one call) and keeps the gradient; backward scales it by the
incoming gradient.  PyTorch only carries the angles and the gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B


class EAEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, handle, dops, terms, f_min, eta_rel):
        p = params.detach().to("cpu", torch.float64).numpy()
        E, g, lnP = B.mps_energy_grad(handle, dops, p, terms, f_min, eta_rel)
        ctx.save_for_backward(torch.from_numpy(np.asarray(g).reshape(p.shape)))
        ctx.lnP = lnP
        return params.new_tensor(E)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g.to(grad_out.device, grad_out.dtype), None, None, None, None, None


def ea_energy(params, state, dops, terms, f_min=1.0, eta_rel=B.ETA_REL_DEFAULT):
    """Differentiable E(params) for an ``EAState`` ``state``."""
    return EAEnergy.apply(params, state.h, dops, terms, f_min, eta_rel)
