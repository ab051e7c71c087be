"""The half-stencil forward (Newton's third law for the pair test): each
unordered pair is tested once by the particle whose upper stencil half holds
the other, and the partner reads the recorded bit.  Its pair set is the full
stencil's, so every operator's forward must match the oracle (and the plain
kernels within rounding) on the parity boxes where it applies, at the benched
grid, with overflowing rows, on a batch and in a graph; its records must never
be replayed as full-stencil records."""
import numpy as np
import pytest
import torch

import oracle
import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import TOL_F32, TOL_F64, box_of, check_close, to_dev
from test_gpu_parity import CASES, OPS, make_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.set_variant(-1)
    c.close()


def variant(word):
    return next(v for v in range(A.variant_count()) if word in A.variant_name(v))


HALF = "half stencil"
MASK = "records accepted-pair bit masks"
PLAIN = "adjoint evaluated on every candidate"


def fwd(ctx, cells, op, params, a_d, v):
    ctx.set_variant(v)
    try:
        return A.pair_sum(ctx, cells, op, params, a_d)
    finally:
        ctx.set_variant(-1)


def wide(g, reach_x=1):
    return int(g.n[0]) >= 2 * reach_x + 1


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_half_stencil_matches_the_oracle(ctx, case):
    g, x, box, prec = make_case(case)
    n, d = x.shape
    print("case", case[0], flush=True)
    cells = A.build_cells(ctx, to_dev(x), [box])
    if not wide(g):
        with pytest.raises(A.AboriaError) as e:
            fwd(ctx, cells, "count", (), None, variant(HALF))
        assert e.value.status == "INVALID_ARG"
        return
    rng = syn.SplitMix64(9191)
    a = (0.2 + 0.3 * rng.uniform(n)).astype(x.dtype).reshape(n, 1)
    a_d = to_dev(a)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    uniform = slice(0, n - n // 5)  # the generated points before the near-boundary ones
    for op, params in OPS:
        aa = a if op == "dem_spring" else None
        aa_d = a_d if op == "dem_spring" else None
        y1 = fwd(ctx, cells, op, params, aa_d, variant(HALF))
        y2 = fwd(ctx, cells, op, params, aa_d, variant(HALF))
        y_plain = fwd(ctx, cells, op, params, aa_d, variant(PLAIN))
        ctx.sync()
        assert torch.equal(y1, y2), (case[0], op)
        if op == "count":
            assert torch.equal(y1, y_plain), case[0]
        yo, so = oracle.pair_sum(g, op, params, x, a=aa)
        check_close(y1.cpu().numpy(), yo, so, tol, "half %s %s" % (case[0], op), normwise=uniform)


def test_headline_grid_and_records(ctx):
    # the spring cube on cells r/3 wide along x: the half forward against the oracle on
    # sampled rows, normwise against the recording forward; the records it leaves are not
    # replayed (a recorded-mask adjoint after it equals the plain adjoint)
    s = syn.spring_cube().systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, [3, 1, 1])
    x_d = to_dev(s.x)
    cells = A.build_cells(ctx, x_d, [box])
    y_half = fwd(ctx, cells, "spring", (1.0,), None, variant(HALF))
    y_mask = fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))
    cnt_half = fwd(ctx, cells, "count", (), None, variant(HALF))
    cnt = fwd(ctx, cells, "count", (), None, variant(PLAIN))
    ctx.sync()
    assert torch.equal(cnt_half, cnt)
    diff = (y_half - y_mask).double().norm().item()
    assert diff <= 1e-6 * y_mask.double().norm().item(), diff
    rows = np.unique(np.floor(syn.SplitMix64(17).uniform(300) * s.n).astype(np.int64))
    g = oracle.grid_of(s, reach=(3, 1, 1))
    yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x, rows=rows, nthreads="all")
    check_close(y_half.cpu().numpy()[rows], yo, so, TOL_F32, "half headline sampled rows")
    gy_d = to_dev(syn.SplitMix64(18).normal(3 * s.n).astype(np.float32).reshape(s.n, 3))
    fwd(ctx, cells, "spring", (1.0,), None, variant(HALF))  # leaves half records behind
    ctx.set_variant(variant(MASK))
    gx_after, _ = A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy_d)
    ctx.set_variant(variant(PLAIN))
    gx_plain, _ = A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy_d)
    ctx.set_variant(-1)
    ctx.sync()
    assert torch.equal(gx_after, gx_plain)
    cells.close()


def test_overflowing_rows_are_tested(ctx):
    # a coarse explicit grid: rows of more than 64 candidates record all ones, and the
    # partner then tests every candidate of such a row
    s = syn.spring_cube(n=40000).systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, [6, 6, 6])
    cells = A.build_cells(ctx, to_dev(s.x), [box])
    y = fwd(ctx, cells, "spring", (1.0,), None, variant(HALF))
    cnt = fwd(ctx, cells, "count", (), None, variant(HALF))
    cnt_ref = fwd(ctx, cells, "count", (), None, variant(PLAIN))
    ctx.sync()
    assert torch.equal(cnt, cnt_ref)
    g = oracle.grid_of(s, ncell=[6, 6, 6])
    yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x)
    check_close(y.cpu().numpy(), yo, so, TOL_F32, "half with overflowing rows")


def test_batch_in_a_graph(ctx):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = A.Context(0, stream)
        w = syn.batch_cubes(nsys=24, nmax=16384)
        xb = np.concatenate([t.x for t in w.systems])
        offsets = np.concatenate([[0], np.cumsum([t.n for t in w.systems])]).tolist()
        boxes = [box_of(t) for t in w.systems]
        x_d = to_dev(xb)
        cells = A.build_cells(gctx, x_d, boxes, offsets)
        gctx.set_variant(variant(HALF))
        y_ref = A.pair_sum(gctx, cells, "spring", (1.0,))
        stream.synchronize()
        y = torch.empty_like(y_ref)
        A.graph_capture_begin(gctx)
        A.build_cells(gctx, x_d, boxes, offsets, cells=cells)
        A.pair_sum(gctx, cells, "spring", (1.0,), y=y)
        graph = A.graph_capture_end(gctx)
        for rep in range(3):
            y.zero_()
            stream.synchronize()
            A.graph_launch(gctx, graph)
            stream.synchronize()
            assert torch.equal(y, y_ref), rep
        graph.close()
        gctx.set_variant(-1)
        gctx.sync()
        for b in (0, 11, 23):
            t = w.systems[b]
            lo, hi = offsets[b], offsets[b + 1]
            yo, so = oracle.pair_sum(oracle.grid_of(t), "spring", (1.0,), t.x)
            check_close(y_ref.cpu().numpy()[lo:hi], yo, so, TOL_F32, "half batch system %d" % b)
        cells.close()
        gctx.close()
