"""The per-wave LDS row windows of the lane kernels.  A row is read from LDS only
when the runs of all lanes of the wave fit one window; denser systems have
rows that do not fit (read from HBM) next to rows that do.  The box search,
the mask-recording forward and its replay must equal, bit for bit, the
recorded-neighbour-list variant, which reads every candidate from HBM, and
the box search must match the oracle."""
import numpy as np
import pytest
import torch

import paper_1704_08907_amd as A
import oracle
from paper_1704_08907_amd import synthetic as syn
from _parity import TOL_F32, box_of, check_close, to_dev

pytestmark = pytest.mark.gpu

MASK = "records accepted-pair bit masks"


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.set_variant(-1)
    c.close()


def variant(word):
    return next(v for v in range(A.variant_count()) if word in A.variant_name(v))


def run(ctx, cells, op, params, gy_d, v):
    ctx.set_variant(v)
    try:
        y = A.pair_sum(ctx, cells, op, params)
        gx, _ = A.pair_sum_backward(ctx, cells, op, params, gy_d)
        return y, gx
    finally:
        ctx.set_variant(-1)


# mean neighbours within r: 30 (every row fits a window), 120 (some rows fit,
# some do not), 220 (rows of 64 lanes span more slots than a window holds)
@pytest.mark.parametrize("neighbours", [30.0, 120.0, 220.0])
@pytest.mark.parametrize("reach", [[1, 1, 1], [3, 1, 1]])
def test_windowed_rows_equal_rows_read_from_hbm(ctx, neighbours, reach):
    w = syn.periodic_cube(12000, neighbours, 31, "spring", (1.0,), "window_cube")
    s = w.systems[0]
    print("neighbours", neighbours, "reach", reach, flush=True)
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, reach)
    cells = A.build_cells(ctx, to_dev(s.x), [box])
    assert A.build_neighbours(ctx, cells, 512) == 512
    rng = syn.SplitMix64(77)
    gy_d = to_dev(rng.normal(s.n * 3).astype(np.float32).reshape(s.n, 3))
    listed = next(v for v in range(A.variant_count()) if "recorded" in A.variant_name(v))
    for op, params in (("spring", (1.0,)), ("soft_sphere", ())):
        g = gy_d if op == "spring" else gy_d[:, :1].contiguous()
        ref = run(ctx, cells, op, params, g, listed)
        box_search = run(ctx, cells, op, params, g, 0)
        masks = run(ctx, cells, op, params, g, variant(MASK))
        fused = A.pair_sum_and_backward(ctx, cells, op, params, g)
        ctx.sync()
        for got in (box_search, masks, fused[:2]):
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), (neighbours, reach, op)
    # the box search against the oracle on every row
    g_or = oracle.grid(3, s.lo, s.hi, s.periodic, s.cutoff, "f32", None, reach)
    y, gx = run(ctx, cells, "spring", (1.0,), gy_d, 0)
    yo, so = oracle.pair_sum(g_or, "spring", (1.0,), s.x.astype(np.float64))
    check_close(y.cpu().numpy(), yo, so, TOL_F32, "window forward %g %s" % (neighbours, reach), normwise=slice(None))
