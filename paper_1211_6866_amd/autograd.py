"""torch.autograd.Function around sai_solve / sai_backward.

forward(A_val, b) splits A (given by its CSR structure and values), builds M
on A~ and returns x = A^{-1} b via Procedure *.  backward(dL/dx) solves the
adjoint system through the transposed split (A^T = A~^T + V U^T) with M^T as
preconditioner and returns dL/dA_val (A's CSR order) and dL/db.  The split
and M depend on the sparsity pattern and are not differentiated.
"""
from __future__ import annotations

import torch


class SAISolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_val, b, row_ptr, col_idx, build_kw: dict, solve_kw: dict):
        from . import Precond, Split, solve
        sp = Split(row_ptr, col_idx, a_val.detach().contiguous())
        pc = Precond(sp, **build_kw)
        x, stats = solve(sp, pc, b.detach().contiguous(), **solve_kw)
        ctx.sp, ctx.pc, ctx.solve_kw = sp, pc, solve_kw
        ctx.stats = stats
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        from . import backward
        (x,) = ctx.saved_tensors
        gb, ga, _ = backward(ctx.sp, ctx.pc, x, grad_x.contiguous(), **ctx.solve_kw)
        return ga, gb, None, None, None, None
