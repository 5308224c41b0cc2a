"""torch.autograd.Function around sai_solve_y / sai_backward_y.

forward(A_val, b) splits A (given by its CSR structure and values), builds M
on A~ and returns x = A^{-1} b via Procedure *, keeping the Krylov solutions
[y, W].  backward(dL/dx) solves the adjoint system A^T lambda = dL/dx through
the transposed split with M^T as preconditioner, one system with A~^T per
correction pass, using the forward's W = A~^{-1} U in
A^{-T} = A~^{-T} (I - V K^{-T} W^T), and returns dL/dA_val (A's CSR order)
and dL/db.  The split and M depend on the sparsity pattern and are not
differentiated.
"""
from __future__ import annotations

import torch


class SAISolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_val, b, row_ptr, col_idx, build_kw: dict, solve_kw: dict):
        from . import Precond, Split, solve_y
        sp = Split(row_ptr, col_idx, a_val.detach().contiguous())
        pc = Precond(sp, **build_kw)
        x, Y, stats = solve_y(sp, pc, b.detach().contiguous(), **solve_kw)
        ctx.sp, ctx.pc, ctx.solve_kw = sp, pc, solve_kw
        ctx.stats = stats
        ctx.save_for_backward(x, Y)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        from . import backward_y
        x, Y = ctx.saved_tensors
        gb, ga, _ = backward_y(ctx.sp, ctx.pc, x, Y, grad_x.contiguous(), **ctx.solve_kw)
        return ga, gb, None, None, None, None
