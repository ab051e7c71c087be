"""GPU parity of the recorded neighbour lists (aboria_build_neighbours).

The replayed forward and adjoint are compared with the oracle (same rules as
the box-search sums) and, bit for bit, with the box-search lane kernels: the
replay adds the same summands in the same order.  Also covered: lists that
overflow their capacity, a list made stale by a rebuild, batches, graph
capture and the argument errors.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import TOL_F32, box_of, check_close, dev, to_dev
from test_gpu_parity import CASES, OPS, make_case, tol_of

pytestmark = pytest.mark.gpu

SEARCH = 0  # lane per particle, box search, summands in box-search order


def replay_variant():
    return next(v for v in range(A.variant_count()) if "recorded" in A.variant_name(v))


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.set_variant(-1)
    c.close()


def inputs(op, n, d, dtype, seed=99):
    rng = syn.SplitMix64(seed)
    a = (0.2 + 0.3 * rng.uniform(n)).astype(dtype).reshape(n, 1) if op == "dem_spring" else None
    ny = A.op_ny(op, d)
    gy = rng.normal(n * ny).astype(dtype).reshape(n, ny)
    return a, gy


def run(ctx, cells, op, params, a_d, gy_d, variant):
    ctx.set_variant(variant)
    try:
        y = A.pair_sum(ctx, cells, op, params, a_d)
        gx, ga = A.pair_sum_backward(ctx, cells, op, params, gy_d, a_d)
    finally:
        ctx.set_variant(-1)
    return y, gx, ga


def same(u, v):
    return (u is None and v is None) or torch.equal(u, v)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("op,params", OPS, ids=[o[0] for o in OPS])
def test_replay_matches_oracle_and_box_search(ctx, case, op, params):
    g, x, box, prec = make_case(case)
    n, d = x.shape
    print("case", case[0], op, flush=True)
    a, gy = inputs(op, n, d, x.dtype)
    cells = A.build_cells(ctx, to_dev(x), [box])
    cap = A.build_neighbours(ctx, cells)
    assert cap >= 8
    a_d = to_dev(a) if a is not None else None
    gy_d = to_dev(gy)
    y, gx, ga = run(ctx, cells, op, params, a_d, gy_d, replay_variant())
    ys, gxs, gas = run(ctx, cells, op, params, a_d, gy_d, SEARCH)
    ctx.sync()
    assert torch.equal(y, ys) and torch.equal(gx, gxs) and same(ga, gas)
    x64 = x.astype(np.float64)
    yo, so = oracle.pair_sum(g, op, params, x64, a=a)
    gxo, gao, sxo, sao = oracle.pair_sum_backward(g, op, params, x64, gy, a=a)
    if op == "count":
        np.testing.assert_array_equal(y.cpu().numpy()[:, 0], yo[:, 0])
        assert torch.all(gx == 0)
        return
    uni = slice(0, n - n // 5)  # the uniform rows of make_case
    check_close(y.cpu().numpy(), yo, so, tol_of(prec), "forward " + op, normwise=uni)
    check_close(gx.cpu().numpy(), gxo, sxo, tol_of(prec), "adjoint " + op, normwise=uni)
    if op == "dem_spring":
        check_close(ga.cpu().numpy(), gao.reshape(-1, 1), sao, tol_of(prec), "adjoint a", normwise=uni)


@pytest.mark.parametrize("capacity", [1, 4, 29])
def test_overflowing_lists_fall_back_to_the_box_search(ctx, capacity):
    w = syn.spring_cube(40000)
    s = w.systems[0]
    print("capacity", capacity, flush=True)
    a, gy = inputs("dem_spring", s.n, 3, np.float32, seed=5)
    cells = A.build_cells(ctx, to_dev(s.x), [box_of(s)])
    assert A.build_neighbours(ctx, cells, capacity) == capacity
    a_d, gy_d = to_dev(a), to_dev(gy)
    for op, params in [("spring", (1.0,)), ("dem_spring", (1.5,)), ("exp_force", (0.7,))]:
        got = run(ctx, cells, op, params, a_d if op == "dem_spring" else None, gy_d, replay_variant())
        ref = run(ctx, cells, op, params, a_d if op == "dem_spring" else None, gy_d, SEARCH)
        ctx.sync()
        for u, v in zip(got, ref):
            assert same(u, v), op


def test_stale_list_after_rebuild_is_not_used(ctx):
    w = syn.spring_cube(50000)
    s = w.systems[0]
    x0 = to_dev(s.x)
    L = float(s.hi[0])
    x1 = torch.remainder(x0 + 0.37, L)
    x1 = torch.where(x1 >= L, torch.zeros_like(x1), x1)
    gy_d = to_dev(inputs("spring", s.n, 3, np.float32)[1])
    cells = A.build_cells(ctx, x0, [box_of(s)])
    A.build_neighbours(ctx, cells)
    A.build_cells(ctx, x1, [box_of(s)], cells=cells)  # the list now describes x0
    y_stale = A.pair_sum(ctx, cells, "spring", (1.0,))
    gx_stale, _ = A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy_d)
    fresh = A.build_cells(ctx, x1.clone(), [box_of(s)])
    y_ref, gx_ref, _ = run(ctx, fresh, "spring", (1.0,), None, gy_d, SEARCH)
    ctx.sync()
    assert torch.equal(y_stale, y_ref) and torch.equal(gx_stale, gx_ref)
    A.build_neighbours(ctx, cells)
    y_new = A.pair_sum(ctx, cells, "spring", (1.0,))
    ctx.sync()
    assert torch.equal(y_new, y_ref)


def test_batch_replay_matches_box_search(ctx):
    w = syn.batch_cubes(nsys=40, nmax=16384)
    xs_all = np.concatenate([s.x for s in w.systems])
    offsets = np.concatenate([[0], np.cumsum([s.n for s in w.systems])]).tolist()
    boxes = [box_of(s) for s in w.systems]
    n = xs_all.shape[0]
    a, gy = inputs("dem_spring", n, 3, np.float32, seed=11)
    cells = A.build_cells(ctx, to_dev(xs_all), boxes, offsets)
    A.build_neighbours(ctx, cells)
    a_d, gy_d = to_dev(a), to_dev(gy)
    for op, params in OPS:
        got = run(ctx, cells, op, params, a_d if op == "dem_spring" else None, gy_d, replay_variant())
        ref = run(ctx, cells, op, params, a_d if op == "dem_spring" else None, gy_d, SEARCH)
        ctx.sync()
        for u, v in zip(got, ref):
            assert same(u, v), op
    # against the oracle, system by system, for the spring
    y_d, gx_d, _ = run(ctx, cells, "spring", (1.0,), None, to_dev(gy[:, :3]), replay_variant())
    ctx.sync()
    y_np, gx_np = y_d.cpu().numpy(), gx_d.cpu().numpy()
    for b in (0, 17, 39):
        s = w.systems[b]
        lo, hi = offsets[b], offsets[b + 1]
        g = oracle.grid_of(s)
        yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x)
        check_close(y_np[lo:hi], yo, so, TOL_F32, "batch forward system %d" % b)
        gxo, _, sxo, _ = oracle.pair_sum_backward(g, "spring", (1.0,), s.x, gy[lo:hi])
        check_close(gx_np[lo:hi], gxo, sxo, TOL_F32, "batch adjoint system %d" % b)


def test_spring_cube_full_size_replay(ctx):
    w = syn.spring_cube()
    s = w.systems[0]
    gy_d = to_dev(w.extra["gy"])
    cells = A.build_cells(ctx, to_dev(s.x), [box_of(s)])
    cap = A.build_neighbours(ctx, cells)
    got = run(ctx, cells, "spring", (1.0,), None, gy_d, replay_variant())
    ref = run(ctx, cells, "spring", (1.0,), None, gy_d, SEARCH)
    cnt = A.pair_sum(ctx, cells, "count", ())
    ctx.sync()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    assert int(cnt.max().item()) <= cap  # no particle needed the fallback


def test_graph_with_neighbour_list_matches_eager():
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = A.Context(0, stream)
        w = syn.spring_cube(30000)
        s = w.systems[0]
        x = to_dev(s.x)
        gy = to_dev(inputs("spring", s.n, 3, np.float32)[1])
        cells = A.build_cells(gctx, x, [box_of(s)])
        A.build_neighbours(gctx, cells)
        y = torch.empty((s.n, 3), device=dev())
        gx = torch.empty((s.n, 3), device=dev())
        A.pair_sum(gctx, cells, "spring", (1.0,), y=y)
        A.pair_sum_backward(gctx, cells, "spring", (1.0,), gy, gx=gx)
        stream.synchronize()
        y_ref, gx_ref = y.clone(), gx.clone()
        A.graph_capture_begin(gctx)
        A.build_cells(gctx, x, [box_of(s)], cells=cells)
        A.build_neighbours(gctx, cells)
        A.pair_sum(gctx, cells, "spring", (1.0,), y=y)
        A.pair_sum_backward(gctx, cells, "spring", (1.0,), gy, gx=gx)
        graph = A.graph_capture_end(gctx)
        for rep in range(3):
            y.zero_()
            gx.zero_()
            stream.synchronize()
            A.graph_launch(gctx, graph)
            stream.synchronize()
            assert torch.equal(y, y_ref), rep
            assert torch.equal(gx, gx_ref), rep
            tmp = A.pair_sum(gctx, cells, "count", ())  # eager work between replays
            stream.synchronize()
            assert tmp.sum().item() > 0
        graph.close()
        gctx.sync()
        gctx.close()


def test_neighbour_list_argument_errors(ctx):
    w = syn.spring_cube(5000)
    s = w.systems[0]
    cells = A.build_cells(ctx, to_dev(s.x), [box_of(s)])
    ctx.set_variant(replay_variant())
    try:
        with pytest.raises(A.AboriaError) as e:
            A.pair_sum(ctx, cells, "spring", (1.0,))
        assert e.value.status == "INVALID_ARG"
    finally:
        ctx.set_variant(-1)
    for bad in (-1, 4097):
        with pytest.raises(A.AboriaError) as e:
            A.build_neighbours(ctx, cells, bad)
        assert e.value.status == "INVALID_ARG"
    assert A.build_neighbours(ctx, cells, 16) == 16
    with pytest.raises(A.AboriaError) as e:
        A.build_neighbours(ctx, cells, 32)  # above the allocated capacity
    assert e.value.status == "INVALID_ARG"
    assert A.build_neighbours(ctx, cells, 8) == 8
    assert A.build_neighbours(ctx, cells) == 16  # automatic: clamped to the allocation
    ctx.sync()
