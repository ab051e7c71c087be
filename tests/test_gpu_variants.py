"""The autotuners: tuned work mappings and tuned cell sizes give results that
match the oracle."""
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


def both(ctx, cells, op, params, a_d, gy_d, v):
    ctx.set_variant(v)
    try:
        y = A.pair_sum(ctx, cells, op, params, a_d)
        gx, ga = A.pair_sum_backward(ctx, cells, op, params, gy_d, a_d)
    finally:
        ctx.set_variant(-1)
    return y, gx, ga


def same(u, v):
    return (u is None and v is None) or torch.equal(u, v)


def test_autotuned_cell_size_gives_valid_coarser_grids(ctx):
    import math

    import oracle
    from _parity import TOL_F32, check_close
    w = syn.batch_cubes(nsys=16, nmax=8192)
    xs_all = np.concatenate([s.x for s in w.systems])
    offsets = np.concatenate([[0], np.cumsum([s.n for s in w.systems])]).tolist()
    boxes = [box_of(s) for s in w.systems]
    x_d = to_dev(xs_all)
    n = xs_all.shape[0]
    for op, params, gy in (("spring", (1.0,), None),
                           ("soft_sphere", (), to_dev(np.ones((n, 1), dtype=np.float32)))):
        tuned, f = A.autotune_cells(ctx, x_d, boxes, offsets, op, params, gy=gy)
        assert f in (1.0, 0.85, 0.7, 0.55)
        for s, t in zip(w.systems, tuned):
            auto = oracle.grid_of(s, None, t.reach).ncell
            assert list(t.ncell) == [max(1, math.floor(f * a)) for a in auto]
        cells = A.build_cells(ctx, x_d, tuned, offsets)
        y = A.pair_sum(ctx, cells, "spring", (1.0,))
        cnt = A.pair_sum(ctx, cells, "count", ())
        ctx.sync()
        for b in (0, 7, 15):
            s, t = w.systems[b], tuned[b]
            g = oracle.grid(3, s.lo, s.hi, s.periodic, s.cutoff, "f32", list(t.ncell), t.reach)
            lo, hi = offsets[b], offsets[b + 1]
            yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x)
            check_close(y.cpu().numpy()[lo:hi], yo, so, TOL_F32, "tuned grid system %d" % b)
            co, _ = oracle.pair_sum(g, "count", (), s.x)
            np.testing.assert_array_equal(cnt.cpu().numpy()[lo:hi, 0], co[:, 0])


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_forward_and_adjoint_equal_the_two_calls(ctx, case):
    g, x, box, prec = make_case(case)
    n, d = x.shape
    cells = A.build_cells(ctx, to_dev(x), [box])
    rng = syn.SplitMix64(6160)
    a_d = to_dev((0.2 + 0.3 * rng.uniform(n)).astype(x.dtype).reshape(n, 1))
    for op, params in OPS:
        gy_d = to_dev(rng.normal(n * A.op_ny(op, d)).astype(x.dtype).reshape(n, -1))
        aa = a_d if op == "dem_spring" else None
        ref = both(ctx, cells, op, params, aa, gy_d, 0)
        got = A.pair_sum_and_backward(ctx, cells, op, params, gy_d, aa)
        ctx.sync()
        for u, v in zip(got, ref):
            assert same(u, v), (case[0], op)


def test_fused_on_a_batch_and_errors(ctx):
    w = syn.batch_cubes(nsys=24, nmax=8192)
    xs_all = np.concatenate([s.x for s in w.systems])
    offsets = np.concatenate([[0], np.cumsum([s.n for s in w.systems])]).tolist()
    cells = A.build_cells(ctx, to_dev(xs_all), [box_of(s) for s in w.systems], offsets)
    n = xs_all.shape[0]
    gy_d = to_dev(np.ones((n, 1), dtype=np.float32))
    ref = both(ctx, cells, "soft_sphere", (), None, gy_d, 0)
    got = A.pair_sum_and_backward(ctx, cells, "soft_sphere", (), gy_d)
    ctx.sync()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    with pytest.raises(A.AboriaError) as e:
        A.pair_sum_and_backward(ctx, cells, "soft_sphere", (), gy_d, y=gy_d)  # y aliases gy
    assert e.value.status == "INVALID_ARG"


def test_tuning_persists_across_contexts(tmp_path):
    # ABORIA_TUNE_CACHE: a context stores its tuning choices in the file, and a new
    # context loads them (the same variant selected without tuning again; the cell-size
    # tuner answers from the cache)
    import json
    import os
    path = str(tmp_path / "tune.json")
    old = os.environ.get("ABORIA_TUNE_CACHE")
    os.environ["ABORIA_TUNE_CACHE"] = path
    try:
        w = syn.spring_cube(n=60000)
        s = w.systems[0]
        x_d = to_dev(s.x)
        c1 = A.Context(0)
        boxes, f = A.autotune_cells(c1, x_d, [box_of(s)], [0, s.n], "spring", (1.0,))
        cells = A.build_cells(c1, x_d, boxes)
        v_f = A.autotune(c1, cells, "spring", (1.0,))
        c1.sync()
        doc = json.load(open(path))
        assert doc["format"] == 1 and doc["arch"]
        assert A.variant_name(v_f) in [e["variant"] for e in doc["variants"]]
        assert len(doc["cells"]) == 1
        c2 = A.Context(0)
        cells2 = A.build_cells(c2, x_d, boxes)
        assert A.selected_variant(c2, cells2, "spring") == v_f
        boxes2, f2 = A.autotune_cells(c2, x_d, [box_of(s)], [0, s.n], "spring", (1.0,))
        assert f2 == f and [b.reach_list() for b in boxes2] == [b.reach_list() for b in boxes]
        assert [list(b.ncell) for b in boxes2] == [list(b.ncell) for b in boxes]
        c2.sync()
        # a forced variant wins over the cache
        other = next(v for v in range(A.variant_count()) if v != v_f and "bit masks" not in A.variant_name(v)
                     and "recorded neighbour list" not in A.variant_name(v) and "all particles" not in A.variant_name(v))
        c2.set_variant(other)
        assert A.selected_variant(c2, cells2, "spring") == other
        c2.set_variant(-1)
        for c in (c1, c2):
            c.close()
    finally:
        if old is None:
            os.environ.pop("ABORIA_TUNE_CACHE", None)
        else:
            os.environ["ABORIA_TUNE_CACHE"] = old


def test_dense_and_build_tuning_persist(tmp_path):
    # the dense launch plan and the radix build shape go to the ABORIA_TUNE_CACHE file
    # too, and a new context uses them without tuning again
    import json
    import os
    path = str(tmp_path / "tune2.json")
    old = os.environ.get("ABORIA_TUNE_CACHE")
    os.environ["ABORIA_TUNE_CACHE"] = path
    try:
        c1 = A.Context(0)
        s = syn.spring_cube(n=60000).systems[0]
        x_d = to_dev(s.x)
        ipt, lb, sh = A.autotune_build(c1, x_d, [box_of(s)])
        rng = syn.SplitMix64(5)
        xt = to_dev(syn.uniform_positions(rng, 3000, [0.0] * 2, [1.0] * 2, "f32"))
        w = to_dev(rng.normal(3000).astype("float32"))
        plan = A.autotune_dense(c1, xt, xt, w, 0.2)
        c1.sync()
        doc = json.load(open(path))
        assert [e["build"] for e in doc["build"]] == [[ipt, lb, sh]]
        name = A.dense_plan_name(plan)
        ti, wg = int(name.split()[0]), int(name.split()[-2])
        assert [e["dense_plan"] for e in doc["dense"]] == [[ti, wg]]
        c2 = A.Context(0)
        cells = A.build_cells(c2, x_d, [box_of(s)])
        v = cells.view()
        assert (v.sort_ipt, v.bucket_bits) == (ipt, lb)  # 2^15 cells: more key bits than any bucket takes
        y2 = A.dense_sum(c2, xt, xt, w, 0.2)
        c2.set_dense_plan(plan)
        y2f = A.dense_sum(c2, xt, xt, w, 0.2)
        torch.cuda.synchronize()
        assert torch.equal(y2, y2f)
        cells.close()
        for c in (c1, c2):
            c.close()
    finally:
        if old is None:
            os.environ.pop("ABORIA_TUNE_CACHE", None)
        else:
            os.environ["ABORIA_TUNE_CACHE"] = old

