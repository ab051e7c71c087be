"""Bit-exact cell lists for the build paths that the small parity cases do not
reach: two radix passes whose position rows travel with the keys (more than
2^20 cells), a tile count too large for the LDS shuffle with a large system
(rows carried), and many small systems (rows gathered), each against the
oracle's cell ids and stable counting sort."""
import numpy as np
import pytest

import oracle
import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import box_of, cells_state, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.close()


def check_system(g, x, keys, perm, off, xs, base_slot=0, base_cell=0):
    ids, st = oracle.cell_ids(g, x)
    assert st == oracle.OK
    operm, ooff = oracle.sort_cells(g, ids)
    n = x.shape[0]
    np.testing.assert_array_equal(perm[base_slot:base_slot + n], operm + base_slot)
    np.testing.assert_array_equal(keys[base_slot:base_slot + n], ids[operm] + base_cell)
    nc = ooff.shape[0] - 1
    np.testing.assert_array_equal(off[base_cell:base_cell + nc + 1], ooff + base_slot)
    np.testing.assert_array_equal(xs[base_slot:base_slot + n, :g.d], x[operm])


@pytest.mark.parametrize("name,n,L", [("two_passes_rows_carried", 300000, 128.0),
                                      ("many_tiles_rows_carried", 2200000, 67.0)])
def test_large_single_system(ctx, name, n, L):
    print(name, flush=True)
    rng = syn.SplitMix64(8080 + n)
    x = syn.uniform_positions(rng, n, [0.0] * 3, [L] * 3, "f32")
    s = syn.System(3, [0.0] * 3, [L] * 3, [1, 1, 1], 1.0, x, "f32")
    g = oracle.grid_of(s)
    cells = A.build_cells(ctx, to_dev(x), [box_of(s)])
    ctx.sync()
    check_system(g, x, *cells_state(cells))
    if name == "two_passes_rows_carried":
        assert int(g.ncells) > (1 << 20)


def test_many_small_systems_rows_gathered(ctx):
    nsys, nb = 64, 40000
    systems, xs_all = [], []
    for b in range(nsys):
        L = syn.side_for_density(nb, 3, 30.0)
        x = syn.uniform_positions(syn.SplitMix64(900 + b), nb, [0.0] * 3, [L] * 3, "f32")
        systems.append(syn.System(3, [0.0] * 3, [L] * 3, [1, 1, 1], 1.0, x, "f32"))
        xs_all.append(x)
    x = np.concatenate(xs_all)
    offsets = [b * nb for b in range(nsys + 1)]
    cells = A.build_cells(ctx, to_dev(x), [box_of(s) for s in systems], offsets)
    ctx.sync()
    keys, perm, off, xs = cells_state(cells)
    base_cell = 0
    for b, s in enumerate(systems):
        g = oracle.grid_of(s)
        if b in (0, 1, 31, 63):
            check_system(g, s.x, keys, perm, off, xs, b * nb, base_cell)
        base_cell += int(g.ncells)


@pytest.mark.parametrize("shuffle", [1, 2])
@pytest.mark.parametrize("ipt", [4, 8, 16])
@pytest.mark.parametrize("low_bits", [8, 9, 10])
def test_every_build_shape_is_bit_exact(ipt, low_bits, shuffle):
    """Every radix build shape the tuner may pick (keys per thread of a sort tile,
    bits sorted per bucket, the scatter's LDS shuffle on or off) gives the
    oracle's cell list, on the spring cube's headline grid (cells r/3 wide along
    x: 158 x 52 x 52, one radix pass or two) and on a batch of uneven systems."""
    sctx = A.Context(0)
    sctx.set_build_shape(ipt, low_bits, shuffle)
    print("build shape", ipt, low_bits, shuffle, flush=True)
    s = syn.spring_cube().systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, [3, 1, 1])
    cells = A.build_cells(sctx, to_dev(s.x), [box])
    cells2 = A.build_cells(sctx, to_dev(s.x), [box], cells=cells)  # a rebuild keeps the shape
    sctx.sync()
    g = oracle.grid_of(s, reach=(3, 1, 1))
    check_system(g, s.x, *cells_state(cells2))
    cells.close()
    w = syn.batch_cubes(nsys=24, nmax=16384)
    xb = np.concatenate([t.x for t in w.systems])
    offsets = np.concatenate([[0], np.cumsum([t.n for t in w.systems])]).tolist()
    cb = A.build_cells(sctx, to_dev(xb), [box_of(t) for t in w.systems], offsets)
    sctx.sync()
    keys, perm, off, xs = cells_state(cb)
    base_cell = 0
    for b, t in enumerate(w.systems):
        gb = oracle.grid_of(t)
        if b in (0, 7, 23):
            check_system(gb, t.x, keys, perm, off, xs, offsets[b], base_cell)
        base_cell += int(gb.ncells)
    cb.close()
    sctx.close()


def test_build_tuner_picks_a_shape_later_builds_use():
    tctx = A.Context(0)
    s = syn.spring_cube(n=1 << 18).systems[0]
    box = box_of(s)
    ipt, lb, sh = A.autotune_build(tctx, to_dev(s.x), [box])
    assert ipt in (4, 8, 16) and 8 <= lb <= 10 and sh in (1, 2)
    cells = A.build_cells(tctx, to_dev(s.x), [box])
    tctx.sync()
    check_system(oracle.grid_of(s), s.x, *cells_state(cells))
    with pytest.raises(A.AboriaError):
        tctx.set_build_shape(5, 0)
    with pytest.raises(A.AboriaError):
        tctx.set_build_shape(0, 11)
    with pytest.raises(A.AboriaError):
        tctx.set_build_shape(0, 0, 3)
    cells.close()
    tctx.close()
