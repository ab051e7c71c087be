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
