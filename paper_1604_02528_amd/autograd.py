"""torch.autograd binding of the selected inversion and its adjoint (float64 and
complex128).

    S = SelInv(n, colptr, rowind, perm, batch=B)
    x, logdet = SelInvFunction.apply(values, S)   # values [B, nnz(A)], requires_grad
    loss = (c * x[:, diag]).sum() + logdet.sum()
    loss.backward()                               # values.grad = dloss/dvalues

x holds the selected entries of A^{-1} on A's stored lower pattern (original
indexing), logdet the log-determinants.  Gradients use the stored-value
convention: an off-diagonal value stands for both (i, j) and (j, i).  The
backward pass hands dloss/dx to the library's scatter (panel layout) and its
reverse sweep (selinv_backward), which also adds the log-det term
d log det A / dA = A^{-1}; no arithmetic happens here.  S holds the buffers of
the last forward call: a backward whose forward is no longer the latest
factorization of S raises instead of differentiating the wrong matrix.

For complex-symmetric A the library's adjoint is the holomorphic one (plain
transposes).  torch passes conjugate cotangents (dL/d conj(y) of a real loss L)
and expects them back for the input, so the binding conjugates gx and glogdet
on the way in and the result on the way out: for a holomorphic map with
Jacobian J that is exactly J^H g.
"""

from __future__ import annotations

import torch

from .selinv import SelInv


class SelInvFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, S: SelInv):
        S.factor(values.detach(), want_dtilde=True)
        S.run()
        x = S.extract()
        logdet = torch.as_tensor(S.logdet(), dtype=S.scalar_dtype, device=x.device)
        ctx.S = S
        ctx.generation = S.generation
        ctx.in_device = values.device
        return x, logdet

    @staticmethod
    def backward(ctx, gx, glogdet):
        S = ctx.S
        if S.generation != ctx.generation:
            raise RuntimeError("SelInvFunction.backward: S was factored again after this forward call; "
                               "run each forward's backward before the next forward on the same SelInv")
        if gx is None:
            gx = torch.zeros((S.batch, S.nnzA), dtype=S.scalar_dtype, device=S.device)
        wl = glogdet
        if S.is_complex:
            gx = gx.conj().resolve_conj()
            wl = None if wl is None else wl.conj().resolve_conj()
        xbar = S.scatter(gx.contiguous())
        abar = S.backward(xbar, None if wl is None else wl.contiguous())
        if S.is_complex:
            abar = abar.conj().resolve_conj()
        return abar.to(ctx.in_device), None
