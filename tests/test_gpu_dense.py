"""GPU parity of the dense kernel sums: the multiquadric kernel of the RBF
example and the adjoint (dL/dw = K^T gy, and the target and source position
gradients) of both kernels, through the C-ABI, against the oracle.  Each
element is compared with the sum of its summands' magnitudes (the scale a
float32 sum's rounding error is bounded by)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1704_08907_amd as A
from paper_1704_08907_amd import synthetic as syn
from _parity import TOL_F32, TOL_F64, to_dev

pytestmark = pytest.mark.gpu

KERNELS = [("gaussian", 0.15), ("multiquadric", 0.2)]


@pytest.fixture(scope="module")
def ctx():
    c = A.Context(0)
    yield c
    c.close()


def inputs(d, prec, nt, ns, seed):
    rng = syn.SplitMix64(seed)
    xt = syn.uniform_positions(rng, nt, [0.0] * d, [1.0] * d, prec)
    xs = syn.uniform_positions(rng, ns, [0.0] * d, [1.0] * d, prec)
    w = rng.normal(ns).astype(xt.dtype)
    gy = rng.normal(nt).astype(xt.dtype)
    return xt, xs, w, gy


def close(got, ref, scale, tol, what):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    err = np.abs(got - ref).max(axis=1)
    bound = tol * np.maximum(scale, 1e-300)
    assert np.all(err <= bound), "%s: worst excess %g (row %d)" % (what, (err - bound).max(), int(np.argmax(err - bound)))


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_multiquadric_forward(ctx, d, prec):
    xt, xs, w, _ = inputs(d, prec, 1000 + 37 * d, 2501, 300 + d)
    y = A.dense_sum(ctx, to_dev(xt), to_dev(xs), to_dev(w), 0.2, kernel="multiquadric")
    yo, so = oracle.dense_sum("multiquadric", 0.2, xt, xs, w)
    close(y.cpu().numpy(), yo, so, TOL_F32 if prec == "f32" else TOL_F64, "multiquadric d=%d" % d)


@pytest.mark.parametrize("kernel,prm", KERNELS, ids=[k[0] for k in KERNELS])
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_backward_all_outputs(ctx, kernel, prm, d, prec):
    xt, xs, w, gy = inputs(d, prec, 1200 + 11 * d, 1700 + 5 * d, 400 + d)
    print("dense backward", kernel, d, prec, flush=True)
    gxt, gxs, gw = A.dense_sum_backward(ctx, to_dev(xt), to_dev(xs), to_dev(w), prm, to_dev(gy), kernel=kernel)
    ref = oracle.dense_backward(kernel, prm, xt, xs, w, gy)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    close(gxt.cpu().numpy(), ref[0], ref[3], tol, "gxt")
    close(gxs.cpu().numpy(), ref[1], ref[4], tol, "gxs")
    close(gw.cpu().numpy(), ref[2], ref[5], tol, "gw")
    # the weight gradient is the forward sum seen from the sources
    yt = A.dense_sum(ctx, to_dev(xs), to_dev(xt), to_dev(gy), prm, kernel=kernel)
    torch.cuda.synchronize()
    assert torch.equal(yt, gw)


def test_backward_full_size_sampled(ctx):
    # the Gaussian workload (N = 65536, sigma = 0.1, float32) with targets = sources;
    # dL/dx = gxt + gxs, checked on sampled rows (the oracle gets the sampled rows as
    # targets for gxt, and as sources for gxs and gw)
    x, w, sigma = syn.gaussian_square()
    n = x.shape[0]
    gy = syn.SplitMix64(12).normal(n).astype(np.float32)
    gxt, gxs, gw = A.dense_sum_backward(ctx, to_dev(x), to_dev(x), to_dev(w), sigma, to_dev(gy))
    rows = np.concatenate([np.floor(syn.SplitMix64(8).uniform(200) * n).astype(np.int64), [0, n - 1]])
    r_gxt = oracle.dense_backward("gaussian", sigma, x[rows], x, w, gy[rows])
    close(gxt.cpu().numpy()[rows], r_gxt[0], r_gxt[3], TOL_F32, "gxt sampled")
    r_src = oracle.dense_backward("gaussian", sigma, x, x[rows], w[rows], gy)
    close(gxs.cpu().numpy()[rows], r_src[1], r_src[4], TOL_F32, "gxs sampled")
    close(gw.cpu().numpy()[rows], r_src[2], r_src[5], TOL_F32, "gw sampled")


def test_backward_in_a_graph_and_edge_cases():
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = A.Context(0, stream)
        xt, xs, w, gy = inputs(2, "f32", 3000, 2000, 77)
        xt_d, xs_d, w_d, gy_d = to_dev(xt), to_dev(xs), to_dev(w), to_dev(gy)
        ref = A.dense_sum_backward(gctx, xt_d, xs_d, w_d, 0.2, gy_d, kernel="multiquadric")
        stream.synchronize()
        outs = [torch.empty_like(t) for t in ref]
        lib = A.lib()
        import ctypes as C
        arr = (C.c_double * 1)(0.2)

        def call():
            st = lib.aboria_dense_sum_backward(gctx.handle, 0, 1, arr, 1, 2, 3000, C.c_void_p(xt_d.data_ptr()),
                                               2000, C.c_void_p(xs_d.data_ptr()), C.c_void_p(w_d.data_ptr()),
                                               C.c_void_p(gy_d.data_ptr()), C.c_void_p(outs[0].data_ptr()),
                                               C.c_void_p(outs[1].data_ptr()), C.c_void_p(outs[2].data_ptr()))
            assert st == 0, gctx.last_error()

        A.graph_capture_begin(gctx)
        call()
        graph = A.graph_capture_end(gctx)
        for rep in range(3):
            for o in outs:
                o.zero_()
            stream.synchronize()
            A.graph_launch(gctx, graph)
            stream.synchronize()
            for o, r in zip(outs, ref):
                assert torch.equal(o, r), rep
        graph.close()
        # no sources: every gradient is zero
        gxt0, gxs0, gw0 = A.dense_sum_backward(gctx, xt_d, xs_d[:0], w_d[:0], 0.2, gy_d)
        stream.synchronize()
        assert torch.all(gxt0 == 0) and gxs0.numel() == 0 and gw0.numel() == 0
        # a non-positive kernel parameter is an argument error
        with pytest.raises(A.AboriaError) as e:
            A.dense_sum_backward(gctx, xt_d, xs_d, w_d, 0.0, gy_d, kernel="multiquadric")
        assert e.value.status == "INVALID_ARG"
        gctx.sync()
        gctx.close()



@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_every_dense_plan_matches_oracle(prec):
    """Every launch plan of the dense tuner (targets per lane, workgroup target),
    forced in turn, against the oracle, forward and backward, on sizes whose
    target blocks and source splits have ragged ends; then the tuner's choice
    serves plain calls."""
    tctx = A.Context(0)
    xt, xs, w, gy = inputs(3, prec, 5000 + 37, 9000 + 11, 900)
    xt_d, xs_d, w_d, gy_d = to_dev(xt), to_dev(xs), to_dev(w), to_dev(gy)
    tol = TOL_F32 if prec == "f32" else TOL_F64
    yo, so = oracle.dense_sum("gaussian", 0.15, xt, xs, w)
    ref = oracle.dense_backward("gaussian", 0.15, xt, xs, w, gy)
    nplans = 0
    while A.dense_plan_name(nplans):
        nplans += 1
    assert nplans >= 6
    for p in range(nplans):
        name = A.dense_plan_name(p)
        print("dense plan", p, name, prec, flush=True)
        tctx.set_dense_plan(p)  # a float-only plan runs the default one in float64
        y = A.dense_sum(tctx, xt_d, xs_d, w_d, 0.15)
        close(y.cpu().numpy(), yo, so, tol, "forward, plan %s" % name)
        gxt, gxs, gw = A.dense_sum_backward(tctx, xt_d, xs_d, w_d, 0.15, gy_d)
        close(gxt.cpu().numpy(), ref[0], ref[3], tol, "gxt, plan %s" % name)
        close(gxs.cpu().numpy(), ref[1], ref[4], tol, "gxs, plan %s" % name)
        close(gw.cpu().numpy(), ref[2], ref[5], tol, "gw, plan %s" % name)
    tctx.set_dense_plan(-1)
    plan = A.autotune_dense(tctx, xt_d, xs_d, w_d, 0.15)
    planb = A.autotune_dense(tctx, xt_d, xs_d, w_d, 0.15, gy=gy_d)
    assert 0 <= plan < nplans and 0 <= planb < nplans
    tctx.set_dense_plan(plan)
    y_forced = A.dense_sum(tctx, xt_d, xs_d, w_d, 0.15)
    tctx.set_dense_plan(-1)
    y = A.dense_sum(tctx, xt_d, xs_d, w_d, 0.15)  # the cached choice
    torch.cuda.synchronize()
    assert torch.equal(y, y_forced)
    tctx.close()
