"""The mask-recording variant: its forward records, per stencil row, the
candidates it accepted; its adjoint replays them.  Both must equal the plain
lane kernels bit for bit -- after a recording, without one (every particle
falls back to testing its candidates), after a rebuild made the record stale,
when rows overflow the record, on a batch and in a graph."""
import numpy as np
import pytest
import torch

import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import box_of, to_dev
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


MASK = "records accepted-pair bit masks"
PLAIN = "adjoint evaluated on every candidate"


def fwd(ctx, cells, op, params, a_d, v):
    ctx.set_variant(v)
    try:
        return A.pair_sum(ctx, cells, op, params, a_d)
    finally:
        ctx.set_variant(-1)


def bwd(ctx, cells, op, params, gy_d, a_d, v):
    ctx.set_variant(v)
    try:
        return A.pair_sum_backward(ctx, cells, op, params, gy_d, a_d)
    finally:
        ctx.set_variant(-1)


def same(u, v):
    return (u is None and v is None) or torch.equal(u, v)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_recorded_masks_equal_the_plain_kernels(ctx, case):
    g, x, box, prec = make_case(case)
    n, d = x.shape
    print("case", case[0], flush=True)
    cells = A.build_cells(ctx, to_dev(x), [box])
    rng = syn.SplitMix64(8080)
    a_d = to_dev((0.2 + 0.3 * rng.uniform(n)).astype(x.dtype).reshape(n, 1))
    for op, params in OPS:
        gy_d = to_dev(rng.normal(n * A.op_ny(op, d)).astype(x.dtype).reshape(n, -1))
        aa = a_d if op == "dem_spring" else None
        y_ref = fwd(ctx, cells, op, params, aa, variant(PLAIN))
        g_ref = bwd(ctx, cells, op, params, gy_d, aa, variant(PLAIN))
        y = fwd(ctx, cells, op, params, aa, variant(MASK))   # records
        g = bwd(ctx, cells, op, params, gy_d, aa, variant(MASK))  # replays
        ctx.sync()
        assert torch.equal(y, y_ref), (case[0], op)
        for u, v in zip(g, g_ref):
            assert same(u, v), (case[0], op)


def test_without_and_after_a_stale_record(ctx):
    w = syn.spring_cube(n=50000)
    s = w.systems[0]
    box = box_of(s)
    x = s.x.copy()
    cells = A.build_cells(ctx, to_dev(x), [box])
    n = x.shape[0]
    gy_d = to_dev(syn.SplitMix64(4).normal(3 * n).astype(np.float32).reshape(n, 3))
    # no record yet: every particle tests its candidates again
    g0 = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(MASK))
    r0 = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(PLAIN))
    assert torch.equal(g0[0], r0[0])
    fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))
    # move the points and rebuild: the record belongs to the previous build
    rng = syn.SplitMix64(5)
    x2 = (x + 0.3 * (rng.uniform(x.size).reshape(x.shape) - 0.5)).astype(np.float32)
    x2 = np.mod(x2 - np.float32(s.lo[0]), np.float32(s.hi[0] - s.lo[0])).astype(np.float32) + np.float32(s.lo[0])
    x2 = np.minimum(x2, np.nextafter(np.float32(s.hi[0]), np.float32(-np.inf)))
    A.build_cells(ctx, to_dev(x2), [box], cells=cells)
    g1 = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(MASK))
    r1 = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(PLAIN))
    ctx.sync()
    assert torch.equal(g1[0], r1[0])


def test_record_serves_another_operator(ctx):
    # the pair set depends on positions and cutoff only, so one forward's record
    # serves the adjoint of any operator on the same build
    w = syn.spring_cube(n=60000)
    s = w.systems[0]
    cells = A.build_cells(ctx, to_dev(s.x), [box_of(s)])
    n = s.n
    rng = syn.SplitMix64(77)
    a_d = to_dev((0.2 + 0.3 * rng.uniform(n)).astype(np.float32).reshape(n, 1))
    fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))  # records
    for op, params in OPS:
        if op == "spring":
            continue
        gy_d = to_dev(rng.normal(n * A.op_ny(op, 3)).astype(np.float32).reshape(n, -1))
        aa = a_d if op == "dem_spring" else None
        g = bwd(ctx, cells, op, params, gy_d, aa, variant(MASK))
        g_ref = bwd(ctx, cells, op, params, gy_d, aa, variant(PLAIN))
        ctx.sync()
        for u, v in zip(g, g_ref):
            assert same(u, v), op


def test_overflowing_rows_fall_back(ctx):
    # a coarse explicit grid packs ~50 candidates per cell, so rows of three cells hold
    # more than 64 candidates and those particles keep no record
    w = syn.spring_cube(n=40000)
    s = w.systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, [6, 6, 6])
    cells = A.build_cells(ctx, to_dev(s.x), [box])
    n = s.n
    gy_d = to_dev(syn.SplitMix64(6).normal(3 * n).astype(np.float32).reshape(n, 3))
    y = fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))
    g = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(MASK))
    y_ref = fwd(ctx, cells, "spring", (1.0,), None, variant(PLAIN))
    g_ref = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(PLAIN))
    ctx.sync()
    assert torch.equal(y, y_ref) and torch.equal(g[0], g_ref[0])


def test_batch_and_graph():
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = A.Context(0, stream)
    w = syn.batch_cubes(nsys=24, nmax=16384)
    xs_all = np.concatenate([q.x for q in w.systems])
    offsets = np.concatenate([[0], np.cumsum([q.n for q in w.systems])]).tolist()
    boxes = [box_of(q) for q in w.systems]
    x_d = to_dev(xs_all)
    n = xs_all.shape[0]
    gy_d = to_dev(syn.SplitMix64(9).normal(3 * n).astype(np.float32).reshape(n, 3))
    cells = A.build_cells(ctx, x_d, boxes, offsets)
    y_ref = fwd(ctx, cells, "spring", (1.0,), None, variant(PLAIN))
    g_ref = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(PLAIN))
    y = torch.empty_like(y_ref)
    gx = torch.empty_like(g_ref[0])

    def step():
        A.build_cells(ctx, x_d, boxes, offsets, cells=cells)
        ctx.set_variant(variant(MASK))
        A.pair_sum(ctx, cells, "spring", (1.0,), y=y)
        A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy_d, gx=gx)
        ctx.set_variant(-1)

    step()
    ctx.sync()
    assert torch.equal(y, y_ref) and torch.equal(gx, g_ref[0])
    A.graph_capture_begin(ctx)
    step()
    graph = A.graph_capture_end(ctx)
    for _ in range(3):
        y.zero_()  # on the same stream as the graph
        gx.zero_()
        A.graph_launch(ctx, graph)
        ctx.sync()
        assert torch.equal(y, y_ref) and torch.equal(gx, g_ref[0])
    graph.close()
    ctx.close()
    torch.cuda.set_stream(torch.cuda.default_stream())


@pytest.mark.parametrize("reach", [[2, 1, 1], [3, 1, 1]])
def test_masks_with_reach_along_x(ctx, reach):
    # narrower cells along x make each of the nine rows a longer run of cells
    w = syn.spring_cube(n=60000)
    s = w.systems[0]
    cells = A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, reach)])
    n = s.n
    rng = syn.SplitMix64(99)
    a_d = to_dev((0.2 + 0.3 * rng.uniform(n)).astype(np.float32).reshape(n, 1))
    for op, params in OPS:
        gy_d = to_dev(rng.normal(n * A.op_ny(op, 3)).astype(np.float32).reshape(n, -1))
        aa = a_d if op == "dem_spring" else None
        y_ref = fwd(ctx, cells, op, params, aa, variant(PLAIN))
        g_ref = bwd(ctx, cells, op, params, gy_d, aa, variant(PLAIN))
        y = fwd(ctx, cells, op, params, aa, variant(MASK))
        g = bwd(ctx, cells, op, params, gy_d, aa, variant(MASK))
        ctx.sync()
        assert torch.equal(y, y_ref), (reach, op)
        for u, v in zip(g, g_ref):
            assert same(u, v), (reach, op)


def test_masks_with_reach_along_x_on_narrow_grids(ctx):
    # fewer than 2m + 1 cells along x: each offset is its own piece of the row
    from test_gpu_reach import NARROW_ANISO, make_case
    for case in NARROW_ANISO:
        g, x, box, prec = make_case(case, [2, 1, 1])
        n, d = x.shape
        cells = A.build_cells(ctx, to_dev(x), [box])
        rng = syn.SplitMix64(5150)
        for op, params in OPS:
            if op == "dem_spring":
                continue
            gy_d = to_dev(rng.normal(n * A.op_ny(op, d)).astype(x.dtype).reshape(n, -1))
            y_ref = fwd(ctx, cells, op, params, None, variant(PLAIN))
            g_ref = bwd(ctx, cells, op, params, gy_d, None, variant(PLAIN))
            y = fwd(ctx, cells, op, params, None, variant(MASK))
            gg = bwd(ctx, cells, op, params, gy_d, None, variant(MASK))
            ctx.sync()
            assert torch.equal(y, y_ref), (case[0], op)
            assert torch.equal(gg[0], g_ref[0]), (case[0], op)


def test_headline_configuration_full_size(ctx):
    # the bench's step: spring cube N = 2^20 on cells r/3 wide along x, the forward
    # recording masks and the adjoint replaying them: the cell list bit-equal to the
    # oracle's, the pair counts of every row bit-equal, the forward and the adjoint of
    # every row against the oracle (threads over rows), and both bit-equal to the row
    # search on the same grid
    import oracle
    from _parity import TOL_F32, cells_state, check_close
    w = syn.spring_cube()
    s = w.systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, [3, 1, 1])
    x_d = to_dev(s.x)
    gy_d = to_dev(w.extra["gy"])
    print("headline full size", flush=True)
    cells = A.build_cells(ctx, x_d, [box])
    assert [int(cells.view().ncell_host[k]) for k in range(3)] == [158, 52, 52]
    y = fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))
    gx = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(MASK))[0]
    cnt = fwd(ctx, cells, "count", (), None, variant(PLAIN))
    y_ref = fwd(ctx, cells, "spring", (1.0,), None, variant(PLAIN))
    gx_ref = bwd(ctx, cells, "spring", (1.0,), gy_d, None, variant(PLAIN))[0]
    ctx.sync()
    assert torch.equal(y, y_ref) and torch.equal(gx, gx_ref)
    g = oracle.grid(3, s.lo, s.hi, s.periodic, s.cutoff, "f32", None, [3, 1, 1])
    x64 = s.x.astype(np.float64)
    keys, perm, off, xs = cells_state(cells)
    ids, st = oracle.cell_ids(g, x64)
    assert st == oracle.OK
    operm, ooff = oracle.sort_cells(g, ids)
    np.testing.assert_array_equal(perm, operm)
    np.testing.assert_array_equal(off, ooff)
    np.testing.assert_array_equal(xs[:, :3], s.x[operm])
    co = oracle.pair_sum(g, "count", (), x64, scales=False, nthreads="all")
    np.testing.assert_array_equal(cnt.cpu().numpy()[:, 0], co[:, 0])
    yo, so = oracle.pair_sum(g, "spring", (1.0,), x64, nthreads="all")
    r = check_close(y.cpu().numpy(), yo, so, TOL_F32, "headline forward, every row")
    gxo, _, sxo, _ = oracle.pair_sum_backward(g, "spring", (1.0,), x64, w.extra["gy"].astype(np.float64),
                                              nthreads="all")
    rg = check_close(gx.cpu().numpy(), gxo, sxo, TOL_F32, "headline adjoint, every row")
    print("worst row error / bound: forward %.3f, adjoint %.3f" % (r, rg))


def test_benched_batch_step_full_size(ctx):
    # the bench's batch step exactly: 512 uneven systems (5.8 M particles), the cell
    # size tuned for the batch, the spring forward recording the pairs and the
    # soft-sphere adjoint (gy = 1) replaying them; eight systems at full size against
    # the oracle (the smallest, the largest and six drawn at random), the forward and
    # the energy gradient of every row of each
    import oracle
    from _parity import TOL_F32, check_close
    w = syn.batch_cubes()
    xs_all = np.concatenate([q.x for q in w.systems])
    offsets = np.concatenate([[0], np.cumsum([q.n for q in w.systems])]).tolist()
    boxes = [A.BoxSpec(3, q.lo, q.hi, q.periodic, q.cutoff) for q in w.systems]
    x_d = to_dev(xs_all)
    g_d = to_dev(w.extra["gy"])
    print("benched batch", xs_all.shape[0], flush=True)
    boxes, _ = A.autotune_cells(ctx, x_d, boxes, offsets, "spring", (1.0,))
    cells = A.build_cells(ctx, x_d, boxes, offsets)
    y = fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))
    gx = bwd(ctx, cells, "soft_sphere", (), g_d, None, variant(MASK))[0]
    ctx.sync()
    sizes = [q.n for q in w.systems]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    pick |= set(np.floor(syn.SplitMix64(77).uniform(6) * len(sizes)).astype(int).tolist())
    y_h, gx_h = y.cpu().numpy(), gx.cpu().numpy()
    for b in sorted(pick):
        q = w.systems[b]
        lo, hi = offsets[b], offsets[b + 1]
        g = oracle.grid_of(q)
        x64 = q.x.astype(np.float64)
        yo, so = oracle.pair_sum(g, "spring", (1.0,), x64, nthreads="all")
        check_close(y_h[lo:hi], yo, so, TOL_F32, "batch system %d forward" % b)
        go, _, sgo, _ = oracle.pair_sum_backward(g, "soft_sphere", (), x64, np.ones((q.n, 1)), nthreads="all")
        check_close(gx_h[lo:hi], go, sgo, TOL_F32, "batch system %d soft-sphere gradient" % b)


def test_needs_reach_1(ctx):
    s = syn.spring_cube(n=20000).systems[0]
    cells = A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, 2)])
    with pytest.raises(A.AboriaError) as e:
        fwd(ctx, cells, "spring", (1.0,), None, variant(MASK))
    assert e.value.status == "INVALID_ARG"
