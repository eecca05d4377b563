"""The solve as a torch.autograd.Function.

Forward: factor A(values) and solve x = A^{-1} b.  Backward (the adjoint of
the solve): grad_b = A^{-T} g by the transpose solve with the same factors
(U^T then L^T sweeps), and grad_values = -grad_b x^T restricted to A's
pattern (``slu_value_gradient``).  If the handle was refactored with other
values between forward and backward, backward factors the forward's values
again first (the handle then holds them).  Every step runs in the library's
kernels.
"""
from __future__ import annotations

import torch


class SparseSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, B, lu):
        lu.factor(values)
        X = lu.solve(B)
        ctx.lu = lu
        ctx.serial = lu._serial
        ctx.save_for_backward(values, X)
        return X

    @staticmethod
    def backward(ctx, G):
        values, X = ctx.saved_tensors
        lu = ctx.lu
        if lu._serial != ctx.serial:
            lu.factor(values.detach())
        GB = lu.solve_transpose(G.contiguous())
        gvals = lu.value_gradient(GB, X) if ctx.needs_input_grad[0] else None
        return gvals, (GB if ctx.needs_input_grad[1] else None), None
