"""GPU parity of the small-system path: the all-pairs variant (every particle of
a system at its minimum image) and the one-kernel build of single-cell cell
lists, against the oracle and against the box search.  The pair set is the
canonical one, so pair counts agree exactly; sums agree within the usual
tolerance (the summation order differs from the box search)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import TOL_F32, TOL_F64, cells_state, check_close, to_dev

pytestmark = pytest.mark.gpu

OPS = [("count", ()), ("spring", (1.0,)), ("soft_sphere", ()), ("exp_force", (0.7,)), ("dem_spring", (1.5,))]


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.set_variant(-1)
    c.close()


def all_pairs_variant():
    return next(v for v in range(A.variant_count()) if "all particles" in A.variant_name(v))


SMALL = [  # id, d, hi, periodic, r, prec, n, single cell
    ("n1", 2, [1.0, 1.0], [1, 1], 0.3, "f64", 1, True),
    ("n2_close", 2, [1.0, 1.0], [1, 1], 0.3, "f64", 2, True),
    ("n7_d1", 1, [3.0], [1], 0.9, "f32", 7, True),
    ("md_square", 2, [1.0, 1.0], [1, 1], 0.1, "f64", 1000, True),
    ("md_square_cells", 2, [1.0, 1.0], [1, 1], 0.1, "f64", 1000, False),
    ("d3_open", 3, [2.0, 2.5, 3.0], [0, 0, 1], 0.6, "f32", 3000, True),
    ("d3_cap", 3, [10.0, 10.0, 10.0], [1, 1, 1], 1.0, "f32", 16384, False),
]


@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
def test_all_pairs_matches_oracle_and_box_search(ctx, case):
    name, d, hi, per, r, prec, n, single = case
    print("small", name, flush=True)
    rng = syn.SplitMix64(2024 + n)
    x = syn.uniform_positions(rng, n, [0.0] * d, hi, prec)
    if name == "n2_close":
        x = np.array([[0.3, 0.4], [0.4, 0.4]], dtype=x.dtype)
    ncell = [1] * d if single else None
    g = oracle.grid(d, [0.0] * d, hi, per, r, prec, ncell)
    box = A.BoxSpec(d, [0.0] * d, hi, per, r, ncell)
    cells = A.build_cells(ctx, to_dev(x), [box])
    if single:
        keys, perm, off, xs = cells_state(cells)
        assert perm.tolist() == list(range(n)) and off.tolist() == [0, n]
        np.testing.assert_array_equal(xs[:, :d], x)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    a = (0.2 + 0.3 * rng.uniform(n)).astype(x.dtype).reshape(n, 1)
    x64 = x.astype(np.float64)
    for op, params in OPS:
        ny = A.op_ny(op, d)
        gy = rng.normal(n * ny).astype(x.dtype).reshape(n, ny)
        a_d = to_dev(a) if op == "dem_spring" else None
        outs = {}
        for v in (all_pairs_variant(), 0):
            ctx.set_variant(v)
            y = A.pair_sum(ctx, cells, op, params, a_d)
            gx, ga = A.pair_sum_backward(ctx, cells, op, params, to_dev(gy), a_d)
            ctx.set_variant(-1)
            outs[v] = (y, gx, ga)
        ctx.sync()
        y, gx, ga = outs[all_pairs_variant()]
        yo, so = oracle.pair_sum(g, op, params, x64, a=a if op == "dem_spring" else None)
        gxo, gao, sxo, sao = oracle.pair_sum_backward(g, op, params, x64, gy, a=a if op == "dem_spring" else None)
        if op == "count":
            np.testing.assert_array_equal(y.cpu().numpy()[:, 0], yo[:, 0])
            assert torch.equal(outs[0][0], y)
            continue
        nw = n >= 1000  # uniform inputs; a handful of pairs has no meaningful norm
        check_close(y.cpu().numpy(), yo, so, tol, "%s forward %s" % (name, op), normwise=nw)
        check_close(gx.cpu().numpy(), gxo, sxo, tol, "%s adjoint %s" % (name, op), normwise=nw)
        if op == "dem_spring":
            check_close(ga.cpu().numpy(), gao.reshape(-1, 1), sao, tol, "%s adjoint a" % name, normwise=nw)


def test_batch_of_single_cell_systems(ctx):
    sizes = [1, 5, 64, 300, 1000, 2500]
    systems, xs_all = [], []
    for k, n in enumerate(sizes):
        L = 0.4 + 0.1 * k
        rng = syn.SplitMix64(70 + k)
        x = syn.uniform_positions(rng, n, [0.0, 0.0, 0.0], [L, L, L], "f32")
        systems.append((L, x))
        xs_all.append(x)
    x = np.concatenate(xs_all)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    r = 0.15
    boxes = [A.BoxSpec(3, [0.0] * 3, [L] * 3, [1, 1, 1], r, [1, 1, 1]) for L, _ in systems]
    cells = A.build_cells(ctx, to_dev(x), boxes, offsets)
    keys, perm, off, _ = cells_state(cells)
    assert perm.tolist() == list(range(x.shape[0]))
    assert off.tolist() == offsets and keys.tolist() == sum([[b] * n for b, n in enumerate(sizes)], [])
    ctx.set_variant(all_pairs_variant())
    y = A.pair_sum(ctx, cells, "spring", (1.0,))
    ctx.set_variant(-1)
    ctx.sync()
    for b, (L, xb) in enumerate(systems):
        g = oracle.grid(3, [0.0] * 3, [L] * 3, [1, 1, 1], r, "f32", [1, 1, 1])
        yo, so = oracle.pair_sum(g, "spring", (1.0,), xb.astype(np.float64))
        check_close(y.cpu().numpy()[offsets[b]:offsets[b + 1]], yo, so, TOL_F32, "system %d" % b,
                    normwise=xb.shape[0] >= 1000)


def test_single_cell_build_reports_domain_errors(ctx):
    x = np.array([[0.2, 0.3], [1.0, 0.5]])  # x == hi is outside the half-open box
    cells = A.build_cells(ctx, to_dev(x), [A.BoxSpec(2, [0.0, 0.0], [1.0, 1.0], [1, 1], 0.3, [1, 1])])
    with pytest.raises(A.AboriaError) as e:
        ctx.sync()
    assert e.value.status == "DOMAIN"
    del cells
