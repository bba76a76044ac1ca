"""log Z as a differentiable function of the codon and codon-pair weights.

``CdzLogZ.apply(theta1, theta2, handle, aa)`` returns log Z (a 0-d float64
tensor on the device).  Its backward pass is the library's hand-written
adjoint (the outside pass, cdz_backward_dev), so the gradients are exactly
the codon marginals d log Z / d theta1[a][c] = Pr(codon a = c) and the
codon-pair marginals d log Z / d theta2[a][x][y] (paper Section 4c: a
codon's contribution isolated through the middle-base tensor of its codon).
PyTorch only supplies device memory and the stream.
"""
from __future__ import annotations

import torch

from . import binding as B


class CdzLogZ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta1: torch.Tensor, theta2, handle, aa: str):
        if theta1.device.type != "cuda" or theta1.dtype != torch.float64:
            raise TypeError("theta1 must be a float64 CUDA tensor [n_aa, 6]")
        t1 = theta1.detach().contiguous()
        t2 = None if theta2 is None else theta2.detach().to(torch.float64).contiguous()
        logz = B.cdz_forward_dev(handle, aa, t1.data_ptr(), 0 if t2 is None else t2.data_ptr())
        ctx.handle = handle
        ctx.aa = aa
        # the weights of this node: the handle keeps only its last forward
        # pass, which another apply() may have replaced before backward runs
        ctx.t1 = t1.clone()
        ctx.t2 = None if t2 is None else t2.clone()
        ctx.dev = theta1.device
        return torch.tensor(logz, dtype=torch.float64, device=theta1.device)

    @staticmethod
    def backward(ctx, grad):
        m = len(ctx.aa)
        t2 = ctx.t2
        # make the handle hold this node's forward pass (free when it already does)
        B.cdz_forward_dev(ctx.handle, ctx.aa, ctx.t1.data_ptr(), 0 if t2 is None else t2.data_ptr())
        d1 = torch.empty((m, 6), dtype=torch.float64, device=ctx.dev)
        d2 = torch.empty((m, 6, 6), dtype=torch.float64, device=ctx.dev) if t2 is not None else None
        B.cdz_backward_dev(ctx.handle, float(grad), d1.data_ptr(), 0 if d2 is None else d2.data_ptr())
        return d1, d2, None, None


def make_handle(energy, prec: str = "fp32"):
    """A library handle on torch's current stream of the current device."""
    return B.cdz_create(energy, prec, stream=torch.cuda.current_stream().cuda_stream)
