"""torch.autograd.Function around the neighbour sum and its hand-written adjoint.

The forward builds (or rebuilds in place) the cell list of the positions and
evaluates the operator; the backward reuses that cell list -- no pair list is
stored -- and calls the adjoint kernel for dL/dx and, for operators with
per-particle variables, dL/da.  All work runs in the HIP library.

When a gradient is needed, no variant is forced on the context, the cells
search one cell deep in y and z and some system is above the small-N switch,
the pair of calls runs the recorded-mask variant: the forward stores which
candidates it accepted and the backward visits only those.  Its results equal
the default row search's bit for bit.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _native as N


# largest system the library's untuned default sums by testing all pairs
SMALL_N_SWITCH = 2048
_MASK_VARIANT = None


def _mask_variant() -> int:
    global _MASK_VARIANT
    if _MASK_VARIANT is None:
        _MASK_VARIANT = next(v for v in range(N.variant_count()) if "accepted-pair bit masks" in N.variant_name(v))
    return _MASK_VARIANT


def _use_masks(ctx: N.Context, cells: N.Cells) -> bool:
    if getattr(ctx, "forced_variant", -1) != -1:
        return False
    if any(m > 1 for b in cells.boxes for m in b.reach_list()[1:]):
        return False
    off = cells.offsets
    return max(off[i + 1] - off[i] for i in range(len(off) - 1)) > SMALL_N_SWITCH


def _with_variant(ctx: N.Context, v: Optional[int], fn):
    if v is None:
        return fn()
    prev = getattr(ctx, "forced_variant", -1)
    ctx.set_variant(v)
    try:
        return fn()
    finally:
        ctx.set_variant(prev)


class PairSum(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x: torch.Tensor, a: Optional[torch.Tensor], ctx: N.Context, boxes: Sequence[N.BoxSpec],
                offsets, op: str, params: tuple, cells: Optional[N.Cells]):
        xd = x.detach().contiguous()
        cells = N.build_cells(ctx, xd, boxes, offsets, cells)
        ad = a.detach().contiguous() if a is not None else None
        grad = fctx.needs_input_grad[0] or fctx.needs_input_grad[1]
        fctx.variant = _mask_variant() if grad and _use_masks(ctx, cells) else None
        y = _with_variant(ctx, fctx.variant, lambda: N.pair_sum(ctx, cells, op, params, ad))
        fctx.cells = cells
        fctx.build = cells.builds
        fctx.nctx = ctx
        fctx.op = op
        fctx.params = params
        fctx.a = ad
        fctx.want_ga = a is not None and a.requires_grad
        return y

    @staticmethod
    def backward(fctx, gy: torch.Tensor):
        if fctx.cells.builds != fctx.build:
            # the adjoint reads the cell list's sorted positions and permutation: after a
            # rebuild with other positions they no longer belong to this forward
            raise RuntimeError("PairSum backward: the cell list passed to this forward was rebuilt (build %d, "
                               "now %d) before the backward ran; give each forward whose gradient is still "
                               "pending its own Cells" % (fctx.build, fctx.cells.builds))
        gx, ga = _with_variant(fctx.nctx, fctx.variant, lambda: N.pair_sum_backward(
            fctx.nctx, fctx.cells, fctx.op, fctx.params, gy.contiguous(), fctx.a, want_ga=fctx.want_ga))
        return gx, (ga if fctx.want_ga else None), None, None, None, None, None, None


def pair_sum(x: torch.Tensor, ctx: N.Context, boxes: Sequence[N.BoxSpec], op: str, params=(),
             a: Optional[torch.Tensor] = None, offsets=None, cells: Optional[N.Cells] = None) -> torch.Tensor:
    """Differentiable y = sum over neighbours of op's summand (original order).

    A caller-supplied cells is rebuilt in place from x; its backward needs that
    build, so a second forward on the same Cells before the first backward makes
    the first backward raise (give such forwards separate Cells)."""
    return PairSum.apply(x, a, ctx, list(boxes), offsets, op, tuple(params), cells)
