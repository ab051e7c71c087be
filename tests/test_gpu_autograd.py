"""The autograd Function around the neighbour sums: torch.autograd.gradcheck
(float64 central differences of the library's own forward against its
hand-written adjoint) for every vector operator, positions and per-particle
variables, periodic and open boxes.  Positions are drawn so that no pair lies
within 1e-4 of the cutoff, so the finite differences never change the pair set."""
import numpy as np
import pytest
import torch

import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from paper_1704_08907_amd.autograd import pair_sum as diff_pair_sum

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.close()


def clear_of_cutoff(x, L, per, r, margin=1e-4):
    d = x[:, None, :] - x[None, :, :]
    for k in range(x.shape[1]):
        if per[k]:
            d[..., k] -= L[k] * np.round(d[..., k] / L[k])
    s = np.sqrt((d * d).sum(-1))
    return not np.any(np.abs(s - r) < margin)


@pytest.mark.parametrize("d,per", [(2, [1, 1]), (3, [1, 0, 1])])
@pytest.mark.parametrize("op,params", [("spring", (1.3,)), ("exp_force", (0.7,)), ("dem_spring", (0.9,))])
def test_gradcheck(ctx, d, per, op, params):
    L = [1.0] * d
    r = 0.3
    n = 30
    seed = 11
    while True:
        rng = syn.SplitMix64(seed)
        x = syn.uniform_positions(rng, n, [0.0] * d, L, "f64")
        x = 0.1 + 0.8 * x if not all(per) else x  # keep open dimensions away from the walls
        if clear_of_cutoff(x, L, per, r):
            break
        seed += 1
    box = A.BoxSpec(d, [0.0] * d, L, per, r)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda:0", requires_grad=True)
    a = None
    if op == "dem_spring":
        a = torch.tensor(0.1 + 0.05 * syn.SplitMix64(3).uniform(n), dtype=torch.float64,
                         device="cuda:0").reshape(n, 1).requires_grad_(True)

    def f(xx, aa=None):
        return diff_pair_sum(xx, ctx, [box], op, params, a=aa)

    inputs = (xt,) if a is None else (xt, a)
    assert torch.autograd.gradcheck(f, inputs, eps=1e-7, atol=1e-6, rtol=1e-5)
    ctx.sync()


def test_energy_gradient_through_autograd_matches_adjoint(ctx):
    w = syn.soft_sphere_cube(20000)
    s = w.systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff)
    x = torch.tensor(s.x, device="cuda:0", requires_grad=True)
    E = diff_pair_sum(x, ctx, [box], "soft_sphere").sum()
    (gx,) = torch.autograd.grad(E, x)
    cells = A.build_cells(ctx, x.detach(), [box])
    gx2, _ = A.pair_sum_backward(ctx, cells, "soft_sphere", (), torch.ones((s.n, 1), device="cuda:0"))
    ctx.sync()
    assert torch.equal(gx, gx2)


def test_spring_gradient_through_autograd_equals_the_row_search(ctx):
    # above the small-N switch the autograd pair runs the recorded-mask variant; its
    # results equal the plain row search bit for bit, and a forced variant is left alone
    w = syn.spring_cube(n=30000)
    s = w.systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff)
    gy = torch.from_numpy(w.extra["gy"][: s.n]).to("cuda:0")
    x = torch.tensor(s.x, device="cuda:0", requires_grad=True)
    y = diff_pair_sum(x, ctx, [box], "spring", (1.0,))
    (gx,) = torch.autograd.grad(y, x, gy)
    plain = next(v for v in range(A.variant_count()) if "adjoint evaluated on every candidate" in A.variant_name(v))
    cells = A.build_cells(ctx, x.detach(), [box])
    ctx.set_variant(plain)
    try:
        y2 = A.pair_sum(ctx, cells, "spring", (1.0,))
        gx2, _ = A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy)
        x3 = x.detach().clone().requires_grad_(True)
        y3 = diff_pair_sum(x3, ctx, [box], "spring", (1.0,))
        (gx3,) = torch.autograd.grad(y3, x3, gy)
        assert ctx.forced_variant == plain
    finally:
        ctx.set_variant(-1)
    ctx.sync()
    assert torch.equal(y.detach(), y2) and torch.equal(gx, gx2)
    assert torch.equal(y3.detach(), y2) and torch.equal(gx3, gx2)


def test_autograd_on_cells_narrower_along_x(ctx):
    # reach {3, 1, 1}: the autograd pair records masks there too; equal to the row search
    w = syn.spring_cube(n=30000)
    s = w.systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, [3, 1, 1])
    gy = torch.from_numpy(w.extra["gy"][: s.n]).to("cuda:0")
    x = torch.tensor(s.x, device="cuda:0", requires_grad=True)
    y = diff_pair_sum(x, ctx, [box], "spring", (1.0,))
    (gx,) = torch.autograd.grad(y, x, gy)
    plain = next(v for v in range(A.variant_count()) if "adjoint evaluated on every candidate" in A.variant_name(v))
    cells = A.build_cells(ctx, x.detach(), [box])
    ctx.set_variant(plain)
    try:
        y2 = A.pair_sum(ctx, cells, "spring", (1.0,))
        gx2, _ = A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy)
    finally:
        ctx.set_variant(-1)
    ctx.sync()
    assert torch.equal(y.detach(), y2) and torch.equal(gx, gx2)


def test_rebuilt_cells_make_a_pending_backward_raise(ctx):
    # two forwards on one caller-supplied Cells: the second rebuilds it in place from
    # other positions, so the first forward's backward would read the wrong sorted
    # positions and permutation; it raises instead, and the second one is correct
    w = syn.spring_cube(8192)
    s = w.systems[0]
    box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff)
    x1 = torch.from_numpy(s.x).to("cuda:0").requires_grad_(True)
    x2 = torch.from_numpy(s.x[::-1].copy()).to("cuda:0").requires_grad_(True)
    cells = A.build_cells(ctx, x1.detach(), [box])
    gy = torch.from_numpy(w.extra["gy"]).to("cuda:0")
    y1 = diff_pair_sum(x1, ctx, [box], "spring", (1.0,), cells=cells)
    y2 = diff_pair_sum(x2, ctx, [box], "spring", (1.0,), cells=cells)
    with pytest.raises(RuntimeError, match="rebuilt"):
        torch.autograd.grad(y1, x1, gy)
    (g2,) = torch.autograd.grad(y2, x2, gy)
    fresh = A.build_cells(ctx, x2.detach(), [box])
    ref, _ = A.pair_sum_backward(ctx, fresh, "spring", (1.0,), gy)
    ctx.sync()
    assert torch.equal(g2, ref)
