"""Cell grids with search reach 2 and 3 (cells about r/2 or r/3 wide, searched
2 or 3 cells deep), in every dimension or along x only, and the flattened,
pruned box search.

Bit-exact against the oracle: cell ids, permutation, offsets and pair sets on
the reach's grid (points placed within a few ulps of the narrower cell
boundaries, where the pruning margins matter).  Sums within the parity
tolerances.  The flattened kernel keeps the row search's order, so it equals
the row-loop lane kernel bit for bit on every grid, reach 1 included, and the
fused call and a replayed neighbour list equal it too."""
import math
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import TOL_F32, TOL_F64, box_of, cells_state, check_close, gpu_pairs_sorted, to_dev
from test_gpu_parity import CASES, OPS, near_boundary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.set_variant(-1)
    c.close()


def variant(word):
    return next(v for v in range(A.variant_count()) if word in A.variant_name(v))


FLAT = "flattened"
ROWS = "adjoint evaluated on every candidate"


# grids narrower than 2m+1 cells (per-offset pieces, aliasing, dropped second wraps)
NARROW = [
    ("d2_narrow", 2, [2.1, 2.6], [1, 1], 1.0, "f32", [3, 4], 700),
    ("d3_narrow_mixed", 3, [2.2, 2.3, 2.4], [1, 0, 1], 1.0, "f64", [4, 2, 3], 600),
]
REACH_CASES = [c for c in CASES if c[6] is None] + NARROW
# reach along x only: the 3^(d-1) rows of the reach-1 search, each over narrower cells
ANISO = [[2, 1, 1], [3, 1, 1]]
NARROW_ANISO = [
    ("d2_narrow_x", 2, [2.1, 2.6], [1, 1], 1.0, "f32", [3, 2], 700),
    ("d3_narrow_x_mixed", 3, [2.2, 2.3, 2.4], [1, 0, 1], 1.0, "f64", [4, 2, 2], 600),
]
ANISO_CASES = [(c, m) for m in ANISO for c in REACH_CASES if c[6] is None and c[1] > 1] + \
    [(c, m) for m in ANISO[:1] for c in NARROW_ANISO]
ALL_REACH = [(c, m) for m in (2, 3) for c in REACH_CASES] + ANISO_CASES
ALL_IDS = ["%s-%s" % (c[0], m if isinstance(m, int) else "".join(map(str, m))) for c, m in ALL_REACH]


def make_case(case, reach):
    name, d, hi, per, r, prec, ncell, n = case
    if not isinstance(reach, int):
        reach = list(reach[:d])
    g = oracle.grid(d, [0.0] * d, hi, per, r, prec, ncell, reach)
    tag = reach if isinstance(reach, int) else 100 + sum(m << (2 * k) for k, m in enumerate(reach))
    rng = syn.SplitMix64(zlib.crc32(name.encode()) + tag)
    x = syn.uniform_positions(rng, n - n // 4, [0.0] * d, hi, prec)
    xb = near_boundary(rng, g, n // 4, prec)
    x = np.ascontiguousarray(np.concatenate([x, xb]))
    box = A.BoxSpec(d, [0.0] * d, hi, per, r, ncell, reach)
    return g, x, box, prec


def run(ctx, cells, op, params, a_d, gy_d, v):
    ctx.set_variant(v)
    try:
        y = A.pair_sum(ctx, cells, op, params, a_d)
        gx, ga = A.pair_sum_backward(ctx, cells, op, params, gy_d, a_d)
    finally:
        ctx.set_variant(-1)
    return y, gx, ga


def same(u, v):
    return (u is None and v is None) or torch.equal(u, v)


@pytest.mark.parametrize("case,reach", ALL_REACH, ids=ALL_IDS)
def test_reach_cells_and_pairs_bit_exact(ctx, case, reach):
    g, x, box, prec = make_case(case, reach)
    print("case", case[0], "reach", reach, flush=True)
    cells = A.build_cells(ctx, to_dev(x), [box])
    ctx.sync()
    v = cells.view()
    assert [v.ncell_host[k] for k in range(g.d)] == g.ncell
    keys, perm, off, xs = cells_state(cells)
    ids, st = oracle.cell_ids(g, x)
    assert st == oracle.OK
    operm, ooff = oracle.sort_cells(g, ids)
    np.testing.assert_array_equal(perm, operm)
    np.testing.assert_array_equal(off, ooff)
    np.testing.assert_array_equal(xs[:, :g.d], x[operm])
    np.testing.assert_array_equal(gpu_pairs_sorted(ctx, cells), oracle.pairs(g, x.astype(np.float64)))


@pytest.mark.parametrize("case,reach", ALL_REACH, ids=ALL_IDS)
def test_reach_sums_match_oracle_and_row_search(ctx, case, reach):
    g, x, box, prec = make_case(case, reach)
    n, d = x.shape
    print("case", case[0], "reach", reach, flush=True)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    cells = A.build_cells(ctx, to_dev(x), [box])
    rng = syn.SplitMix64(424242)
    a = (0.2 + 0.3 * rng.uniform(n)).astype(x.dtype).reshape(n, 1)
    x64 = x.astype(np.float64)
    for op, params in OPS:
        gy = rng.normal(n * A.op_ny(op, d)).astype(x.dtype).reshape(n, -1)
        aa = a if op == "dem_spring" else None
        aa_d = to_dev(aa) if aa is not None else None
        gy_d = to_dev(gy)
        # the untuned default above the small-N switch: the flattened search at reach > 1 in y
        # or z, the row search otherwise (the two are equal bit for bit)
        y = A.pair_sum(ctx, cells, op, params, aa_d)
        gx, ga = A.pair_sum_backward(ctx, cells, op, params, gy_d, aa_d)
        flat = run(ctx, cells, op, params, aa_d, gy_d, variant(FLAT))
        rows = run(ctx, cells, op, params, aa_d, gy_d, variant(ROWS))
        fused = A.pair_sum_and_backward(ctx, cells, op, params, gy_d, aa_d)  # one search for both
        ctx.sync()
        for u, v in zip(fused, rows):
            assert same(u, v), (case[0], op, "fused")
        if n > 2048:  # smaller systems default to the all-pairs sums
            for u, v in zip((y, gx, ga), flat):
                assert same(u, v), (case[0], op, "default")
        for u, v in zip(rows, flat):
            assert same(u, v), (case[0], op, "row search")
        yo, so = oracle.pair_sum(g, op, params, x64, a=aa)
        gxo, gao, sxo, sao = oracle.pair_sum_backward(g, op, params, x64, gy, a=aa)
        if op == "count":
            np.testing.assert_array_equal(y.cpu().numpy()[:, 0], yo[:, 0])
            continue
        uni = slice(0, n - n // 4)  # the uniform rows (the rest sit within ulps of cell faces)
        check_close(y.cpu().numpy(), yo, so, tol, "forward " + op, normwise=uni)
        check_close(gx.cpu().numpy(), gxo, sxo, tol, "adjoint " + op, normwise=uni)
        if op == "dem_spring":
            check_close(ga.cpu().numpy(), gao.reshape(-1, 1), sao, tol, "adjoint a", normwise=uni)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_flat_equals_row_search_at_reach_1(ctx, case):
    name, d, hi, per, r, prec, ncell, n = case
    g, x, _, _ = make_case((name, d, hi, per, r, prec, ncell, n), 1)
    box = A.BoxSpec(d, [0.0] * d, hi, per, r, ncell)
    print("case", name, flush=True)
    cells = A.build_cells(ctx, to_dev(x), [box])
    rng = syn.SplitMix64(7)
    a_d = to_dev((0.2 + 0.3 * rng.uniform(n)).astype(x.dtype).reshape(n, 1))
    for op, params in OPS:
        gy_d = to_dev(rng.normal(n * A.op_ny(op, d)).astype(x.dtype).reshape(n, -1))
        aa = a_d if op == "dem_spring" else None
        ref = run(ctx, cells, op, params, aa, gy_d, variant(ROWS))
        got = run(ctx, cells, op, params, aa, gy_d, variant(FLAT))
        ctx.sync()
        for u, v in zip(got, ref):
            assert same(u, v), (name, op)


def test_reach_fused_and_replayed_list_equal_the_flat_search(ctx):
    w = syn.spring_cube(n=60000)
    s = w.systems[0]
    box = A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, None, 2)
    x_d = to_dev(s.x)
    cells = A.build_cells(ctx, x_d, [box])
    n = s.x.shape[0]
    gy_d = to_dev(syn.SplitMix64(31).normal(3 * n).astype(np.float32).reshape(n, 3))
    ref = run(ctx, cells, "spring", (1.0,), None, gy_d, variant(FLAT))
    fused = A.pair_sum_and_backward(ctx, cells, "spring", (1.0,), gy_d)
    A.build_neighbours(ctx, cells)
    replay = run(ctx, cells, "spring", (1.0,), None, gy_d, variant("recorded neighbour list"))
    ctx.sync()
    for u, v in zip(fused, ref):
        assert same(u, v)
    for u, v in zip(replay, ref):
        assert same(u, v)
    g = oracle.grid(3, s.lo, s.hi, s.periodic, s.cutoff, "f32", None, 2)
    rows = np.arange(0, n, 150)
    yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x.astype(np.float64), rows=rows)
    check_close(ref[0].cpu().numpy()[rows], yo, so, TOL_F32, "spring cube reach 2 sampled rows")


def test_batch_of_mixed_reaches(ctx):
    w = syn.batch_cubes(nsys=12, nmax=8192)
    reaches = [[[1, 1, 1], [2, 2, 2], [3, 3, 3], [2, 1, 1], [3, 1, 1]][b % 5] for b in range(len(w.systems))]
    xs_all = np.concatenate([s.x for s in w.systems])
    offsets = np.concatenate([[0], np.cumsum([s.n for s in w.systems])]).tolist()
    boxes = [A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, None, m) for s, m in zip(w.systems, reaches)]
    cells = A.build_cells(ctx, to_dev(xs_all), boxes, offsets)
    n = xs_all.shape[0]
    gy = syn.SplitMix64(12).normal(3 * n).astype(np.float32).reshape(n, 3)
    gy_d = to_dev(gy)
    flat = run(ctx, cells, "spring", (1.0,), None, gy_d, variant(FLAT))
    rows = run(ctx, cells, "spring", (1.0,), None, gy_d, variant(ROWS))
    ctx.sync()
    assert torch.equal(flat[0], rows[0]) and torch.equal(flat[1], rows[1])
    for b in (0, 1, 2, 5, 11):
        s = w.systems[b]
        g = oracle.grid(3, s.lo, s.hi, s.periodic, s.cutoff, "f32", None, reaches[b])
        lo, hi = offsets[b], offsets[b + 1]
        yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x.astype(np.float64))
        check_close(flat[0].cpu().numpy()[lo:hi], yo, so, TOL_F32, "system %d forward" % b)
        gxo, _, sxo, _ = oracle.pair_sum_backward(g, "spring", (1.0,), s.x.astype(np.float64), gy[lo:hi])
        check_close(flat[1].cpu().numpy()[lo:hi], gxo, sxo, TOL_F32, "system %d adjoint" % b)


def test_mask_variant_needs_reach_1_in_y_and_z(ctx):
    # the mask record holds the 3^(d-1) rows of the paper's stencil: deeper
    # searches in y or z are refused, and the tuner never picks it alone
    w = syn.spring_cube(n=20000)
    s = w.systems[0]
    cells = A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, None, 2)])
    ctx.set_variant(variant("records accepted-pair bit masks"))
    try:
        with pytest.raises(A.AboriaError) as e:
            A.pair_sum(ctx, cells, "spring", (1.0,))
        assert e.value.status == "INVALID_ARG"
    finally:
        ctx.set_variant(-1)
    choice = A.autotune(ctx, cells, "spring", (1.0,))
    assert "bit masks" not in A.variant_name(choice)
    # reach 2 along x only: the mask variant runs
    cx = A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, None, [2, 1, 1])])
    ctx.set_variant(variant("records accepted-pair bit masks"))
    try:
        A.pair_sum(ctx, cx, "spring", (1.0,))
    finally:
        ctx.set_variant(-1)
    with pytest.raises(A.AboriaError):
        A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, None, 4)])
    with pytest.raises(A.AboriaError):
        A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, None, [1, 4, 1])])
    with pytest.raises(A.AboriaError):  # explicit counts finer than reach 1 allows
        A.build_cells(ctx, to_dev(s.x), [A.BoxSpec(s.d, s.lo, s.hi, s.periodic, s.cutoff, [40, 40, 40], 1)])
    ctx.sync()


def test_autotuned_reach_and_cell_size_are_valid(ctx):
    w = syn.batch_cubes(nsys=8, nmax=16384)
    xs_all = np.concatenate([s.x for s in w.systems])
    offsets = np.concatenate([[0], np.cumsum([s.n for s in w.systems])]).tolist()
    x_d = to_dev(xs_all)
    tuned, f = A.autotune_cells(ctx, x_d, [box_of(s) for s in w.systems], offsets, "spring", (1.0,))
    assert f in (1.0, 0.85, 0.7, 0.55)
    m = tuned[0].reach
    assert m in ([1, 1, 1], [2, 2, 2], [3, 3, 3], [2, 1, 1], [3, 1, 1]) and all(t.reach == m for t in tuned)
    for s, t in zip(w.systems, tuned):
        auto = oracle.grid_of(s, None, m).ncell
        assert list(t.ncell) == [max(1, math.floor(f * a)) for a in auto]
    cells = A.build_cells(ctx, x_d, tuned, offsets)
    y = A.pair_sum(ctx, cells, "spring", (1.0,))
    ctx.sync()
    for b in (0, 7):
        s, t = w.systems[b], tuned[b]
        g = oracle.grid(3, s.lo, s.hi, s.periodic, s.cutoff, "f32", list(t.ncell), m)
        lo, hi = offsets[b], offsets[b + 1]
        yo, so = oracle.pair_sum(g, "spring", (1.0,), s.x.astype(np.float64))
        check_close(y.cpu().numpy()[lo:hi], yo, so, TOL_F32, "tuned system %d" % b)
