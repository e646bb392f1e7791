"""Differentiable triangular solve on a (possibly rewritten) DAG.

Forward: X = L^{-1} B, solved on the rewritten system L' = M L, B' = M B
(equation rewriting, paper Section 2.2), with X kept for the backward pass.
Backward (hand-written adjoint): Y = L'^{-T} G by the transposed solve (the
upper-triangular system, levels in reverse order), grad_B = M^T Y = Y - C^T Y,
and grad_L = -grad_B X^T on the stored pattern of the *original* L.
"""
from __future__ import annotations

import torch

from .api import CSRMatrix, Plan, Rewriter, analyze, apply_MT, grad_vals

__all__ = ["TriangularSolve", "SpTRSVFunction"]


class TriangularSolve:
    """Holds the analysis, the rewrite and the solve plan of one pattern.

    Calling it with (vals, B) returns X = L(vals)^{-1} B, differentiable with
    respect to vals and B.  rows / targets select the rewritten rows (None:
    solve on the original DAG)."""

    def __init__(self, L: CSRMatrix, rows=None, targets=None, algo: str = "auto", kmax: int = 1,
                 **plan_opts):
        # a private copy of the values: the plan solves with whatever this
        # buffer holds, and callers' tensors are never written
        self.L = L.with_vals(L.vals.detach().clone())
        self.info = analyze(self.L)
        self.rw = None
        if rows is not None:
            self.rw = Rewriter(self.L, self.info.level, rows, targets)
            self.rw.numeric(None, None)
            # multipliers of the rewrite; their C^T ordering is built once
            self.rwres = self.rw.result()
            self.plan = Plan(self.rw.Lp, algo=algo, kmax=kmax, **plan_opts)
        else:
            self.plan = Plan(self.L, algo=algo, kmax=kmax, **plan_opts)
        self.kmax = kmax

    def _load(self, vals: torch.Tensor) -> None:
        """Make the plan's matrix hold these values (L, and L' if rewritten)."""
        if not torch.equal(vals, self.L.vals):
            self.L.vals.copy_(vals)
            if self.rw is not None:
                self.rw.numeric(None, None)

    def __call__(self, vals: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        return SpTRSVFunction.apply(vals, B, self)

    # the forward and backward passes as plain functions (no autograd)
    def forward_solve(self, vals: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        self._load(vals)
        if self.rw is not None:
            Bp = self.rw.numeric(None, B)
            return self.plan.solve(Bp)
        return self.plan.solve(B)

    def adjoint(self, X: torch.Tensor, G: torch.Tensor,
                vals: torch.Tensor | None = None) -> tuple[torch.Tensor, torch.Tensor]:
        if vals is not None:
            self._load(vals)
        Y = self.plan.solve_transpose(G.contiguous())
        gB = apply_MT(self.rwres, Y) if self.rw is not None else Y
        gV = grad_vals(self.L, gB, X)
        return gV, gB


class SpTRSVFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, B, solver: TriangularSolve):
        X = solver.forward_solve(vals.detach(), B.detach().contiguous())
        ctx.solver = solver
        ctx.save_for_backward(X, vals.detach())
        return X

    @staticmethod
    def backward(ctx, G):
        X, vals = ctx.saved_tensors
        gV, gB = ctx.solver.adjoint(X, G, vals)
        return gV, gB.reshape(G.shape), None
