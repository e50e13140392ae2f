"""Differentiable PageRank on a fixed sparsity pattern (torch.autograd).

The forward pass is the power method of Sec. 5.5.1 (``Plan.pagerank``) on the
column-normalised edge weights P = w / colsum(w).  The backward pass never
stores iterates: it solves the adjoint fixed point

    lambda = dL/dx* + alpha P^T lambda + (alpha / n) (1^T lambda) d

with the merge-path SpMV of a second plan built on the transpose of the
pattern (``Plan.transpose``), forms dL/dP[e] = alpha lambda[row] x*[col] with
a per-nonzero kernel, and differentiates the column normalisation with a
gather through the transpose's permutation, a transposed SpMV (column sums)
and a column scaling.  Every step is a kernel of libmerbit.so; torch provides
the tensors and the autograd graph only.
"""
from __future__ import annotations

import torch

from .merbit import Plan, column_scale, gather_values


class DiffPageRank:
    """Plans and buffers for PageRank of column-normalised weights on one
    pattern (CSR rows = destinations, columns = sources).

    alpha, tol, max_iter, check_every apply to the forward power method;
    adj_tol / adj_max_iter to the adjoint fixed point (defaults: the same).
    stripes = S > 1 runs the forward power method and the adjoint fixed point
    on column-stripe plans (a second plan of P, and P^T's plan); the plain
    plan of P keeps the transpose and the per-nonzero products.
    """

    def __init__(self, row_ptr: torch.Tensor, col_ind: torch.Tensor, n: int, *,
                 dtype=torch.float32, alpha: float = 0.85, tol: float = 0.0,
                 max_iter: int = 100, check_every: int = 10, adj_tol: float | None = None,
                 adj_max_iter: int | None = None, sigma: int = 0, stripes: int = 0,
                 stream=None):
        dev = col_ind.device
        self.n = int(n)
        self.nnz = col_ind.numel()
        self.dtype = dtype
        self.alpha, self.tol, self.max_iter, self.check_every = alpha, tol, max_iter, check_every
        self.adj_tol = tol if adj_tol is None else adj_tol
        self.adj_max_iter = max_iter if adj_max_iter is None else adj_max_iter
        self.stream = stream
        self.col = col_ind
        self.values = torch.zeros(self.nnz, dtype=dtype, device=dev)  # P, persistent
        self.stripes = stripes if stripes > 1 else 0
        self.plan = Plan(row_ptr, col_ind, self.values, n, sigma=sigma, stream=stream)
        # the forward power method's plan: a column-stripe plan keeps its own
        # copy of the values (refreshed after every write to self.values)
        self.plan_fwd = (Plan(row_ptr, col_ind, self.values, n, sigma=sigma,
                              stripes=self.stripes, stream=stream)
                         if self.stripes else self.plan)
        self.row_t, self.col_t, self.perm = self.plan.transpose(stream=stream)
        self.values_t = torch.zeros(self.nnz, dtype=dtype, device=dev)  # P^T, persistent
        self.plan_t = Plan(self.row_t, self.col_t, self.values_t, n, sigma=sigma,
                           stripes=self.stripes, stream=stream)
        self.ones = torch.ones(n, dtype=dtype, device=dev)
        self.x0 = torch.full((n,), 1.0 / n, dtype=dtype, device=dev)
        # the iterates live in buffers owned here, so every call hands the
        # library the same pointers and its recorded HIP graphs of the
        # iteration chunks replay from one training step to the next; results
        # are copied out
        self.x_work = torch.empty(n, dtype=dtype, device=dev)
        self.g_work = torch.empty(n, dtype=dtype, device=dev)
        self.lam_work = torch.empty(n, dtype=dtype, device=dev)
        self.last_forward = None   # (iterations, l1 change) of the last forward solve
        self.last_adjoint = None

    def refresh_transpose_values(self):
        """After a write to values_t: a column-stripe plan of P^T re-copies them."""
        if self.stripes:
            self.plan_t.set_values(self.values_t)

    # column sums over the pattern's columns of per-nonzero values a[e] (times
    # b[e]): the transpose's SpMV with a vector of ones
    def _column_sums(self, a: torch.Tensor, b: torch.Tensor | None = None) -> torch.Tensor:
        gather_values(self.perm, a, b, out=self.values_t, stream=self.stream)
        self.refresh_transpose_values()
        return self.plan_t.spmv(self.ones, stream=self.stream)

    def colnorm(self, w: torch.Tensor) -> torch.Tensor:
        return _ColumnNormalize.apply(w, self)

    def pagerank(self, P: torch.Tensor) -> torch.Tensor:
        return _PageRank.apply(P, self)

    def __call__(self, w: torch.Tensor) -> torch.Tensor:
        """x*(colnorm(w))."""
        return self.pagerank(self.colnorm(w))

    def close(self):
        if self.plan_fwd is not self.plan:
            self.plan_fwd.close()
        self.plan.close()
        self.plan_t.close()


class _ColumnNormalize(torch.autograd.Function):
    """P[e] = w[e] / s[col(e)], s = column sums of w."""

    @staticmethod
    def forward(ctx, w, op: DiffPageRank):
        w = w.detach().contiguous()
        s = op._column_sums(w)
        P = column_scale(op.col, w, s, stream=op.stream)
        ctx.op = op
        ctx.save_for_backward(P, s)
        return P

    @staticmethod
    def backward(ctx, G):
        op = ctx.op
        P, s = ctx.saved_tensors
        G = G.contiguous().to(op.dtype)
        t = op._column_sums(G, P)            # t[c] = sum over column c of G[e] P[e]
        return column_scale(op.col, G, s, t, stream=op.stream), None


class _PageRank(torch.autograd.Function):
    """x* = fixed point of x -> alpha P x + (alpha d^T x + 1 - alpha) / n."""

    @staticmethod
    def forward(ctx, P, op: DiffPageRank):
        P = P.detach().contiguous()
        op.values.copy_(P)
        if op.plan_fwd is not op.plan:
            op.plan_fwd.set_values(op.values)
        op.x_work.copy_(op.x0)
        it, res, _ = op.plan_fwd.pagerank(op.x_work, op.alpha, op.tol, op.max_iter,
                                          op.check_every, stream=op.stream)
        x = op.x_work.clone()
        op.last_forward = (it, res)
        ctx.op = op
        ctx.save_for_backward(P, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        op = ctx.op
        P, x = ctx.saved_tensors
        gx = gx.contiguous().to(op.dtype)
        gather_values(op.perm, P, out=op.values_t, stream=op.stream)   # P^T's values
        op.refresh_transpose_values()
        op.g_work.copy_(gx)
        op.lam_work.copy_(gx)
        it, res, _ = op.plan.pagerank_adjoint(op.plan_t, op.g_work, op.lam_work, op.alpha,
                                              op.adj_tol, op.adj_max_iter, op.check_every,
                                              stream=op.stream)
        op.last_adjoint = (it, res)
        return op.plan.sddmm(op.lam_work, x, op.alpha, stream=op.stream), None
