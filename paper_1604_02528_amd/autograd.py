"""torch.autograd binding of the selected inversion and its adjoint (FP64).

    S = SelInv(n, colptr, rowind, perm, batch=B)
    x, logdet = SelInvFunction.apply(values, S)   # values [B, nnz(A)], requires_grad
    loss = (c * x[:, diag]).sum() + logdet.sum()
    loss.backward()                               # values.grad = dloss/dvalues

x holds the selected entries of A^{-1} on A's stored lower pattern (original
indexing), logdet the log-determinants.  Gradients use the stored-value
convention: an off-diagonal value stands for both (i, j) and (j, i).  The
backward pass scatters dloss/dx into the panel layout (selinv_scatter) and runs
the library's reverse sweep (selinv_backward); d logdet / da is the selected
inverse itself (doubled off the diagonal).  S keeps the state of the last
forward call, so each forward must be followed by its own backward before S is
used again.
"""

from __future__ import annotations

import numpy as np
import torch

from .selinv import SelInv


def _offdiag_scale(S: SelInv) -> torch.Tensor:
    if getattr(S, "_offdiag", None) is None:
        cols = np.repeat(np.arange(S.n), np.diff(S._colptr))
        scale = np.where(S._rowind == cols, 1.0, 2.0)
        S._offdiag = torch.from_numpy(scale).to(S.device)
    return S._offdiag


class SelInvFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, S):
        if S.is_complex:
            raise NotImplementedError("the adjoint is implemented for float64 only")
        S.factor(values.detach(), want_dtilde=True)
        S.run()
        x = S.extract()
        logdet = torch.as_tensor(S.logdet(), dtype=torch.float64, device=x.device)
        ctx.S = S
        ctx.in_device = values.device
        ctx.save_for_backward(x)
        return x, logdet

    @staticmethod
    def backward(ctx, gx, glogdet):
        S = ctx.S
        (x,) = ctx.saved_tensors
        if gx is None:
            gx = torch.zeros_like(x)
        xbar = S.scatter(gx.contiguous())
        abar = S.backward(xbar)
        if glogdet is not None:
            abar = abar + glogdet.reshape(-1, 1) * x * _offdiag_scale(S)
        return abar.to(ctx.in_device), None
