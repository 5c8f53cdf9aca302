"""torch.autograd wrapper: traces as a differentiable function of the permittivity.

``TracesFn.apply(eps, ctx_obj, acq)`` returns the receiver traces (FP64 tensor
[n_src, n_rec, n_steps]) for the fine-element permittivity ``eps``; its backward pass is
the reverse-time adjoint of libmgrt (``mgrt_misfit_gradient``, level "fine"), i.e. the
exact vector-Jacobian product of the leap-frog scheme (Sec. II-B / App. A-1).  Both
directions run inside the library; this module only moves tensors across the boundary.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch


@dataclass
class Acquisition:
    src: np.ndarray          # (n_src, d)
    rec: np.ndarray          # (n_src, n_rec, d)
    wavelet: np.ndarray      # (n_steps,)
    dt: float
    n_steps: int
    precision: int = 32


class TracesFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, lib_ctx, acq: Acquisition):
        e = eps.detach().cpu().double().numpy()
        lib_ctx.upload_permittivity(e)
        tr = lib_ctx.forward_traces(acq.src, acq.rec, acq.wavelet, acq.dt, acq.n_steps,
                                    precision=acq.precision)
        ctx.lib_ctx = lib_ctx
        ctx.acq = acq
        ctx.eps_np = e
        ctx.device = eps.device
        return torch.from_numpy(tr).to(eps.device)

    @staticmethod
    def backward(ctx, grad_out):
        acq = ctx.acq
        ctx.lib_ctx.upload_permittivity(ctx.eps_np)
        rho = grad_out.detach().cpu().double().numpy()
        g = ctx.lib_ctx.misfit_gradient(acq.src, acq.rec, acq.wavelet, acq.dt, acq.n_steps, rho,
                                        level="fine", precision=acq.precision)
        return torch.from_numpy(g).to(ctx.device), None, None


def traces(eps: torch.Tensor, lib_ctx, acq: Acquisition) -> torch.Tensor:
    """Differentiable traces for fine-element permittivity eps (shape (n_elems,))."""
    return TracesFn.apply(eps, lib_ctx, acq)
