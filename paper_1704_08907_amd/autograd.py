"""torch.autograd.Function around the neighbour sum and its hand-written adjoint.

The forward builds (or rebuilds in place) the cell list of the positions and
evaluates the operator; the backward reuses that cell list -- no pair list is
stored -- and calls the adjoint kernel for dL/dx and, for operators with
per-particle variables, dL/da.  All work runs in the HIP library.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _native as N


class PairSum(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x: torch.Tensor, a: Optional[torch.Tensor], ctx: N.Context, boxes: Sequence[N.BoxSpec],
                offsets, op: str, params: tuple, cells: Optional[N.Cells]):
        xd = x.detach().contiguous()
        cells = N.build_cells(ctx, xd, boxes, offsets, cells)
        ad = a.detach().contiguous() if a is not None else None
        y = N.pair_sum(ctx, cells, op, params, ad)
        fctx.cells = cells
        fctx.nctx = ctx
        fctx.op = op
        fctx.params = params
        fctx.a = ad
        fctx.want_ga = a is not None and a.requires_grad
        return y

    @staticmethod
    def backward(fctx, gy: torch.Tensor):
        gx, ga = N.pair_sum_backward(fctx.nctx, fctx.cells, fctx.op, fctx.params, gy.contiguous(), fctx.a,
                                     want_ga=fctx.want_ga)
        return gx, (ga if fctx.want_ga else None), None, None, None, None, None, None


def pair_sum(x: torch.Tensor, ctx: N.Context, boxes: Sequence[N.BoxSpec], op: str, params=(),
             a: Optional[torch.Tensor] = None, offsets=None, cells: Optional[N.Cells] = None) -> torch.Tensor:
    """Differentiable y = sum over neighbours of op's summand (original order)."""
    return PairSum.apply(x, a, ctx, list(boxes), offsets, op, tuple(params), cells)
