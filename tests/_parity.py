"""Shared helpers of the GPU parity tests (comparison rules and converters)."""
import numpy as np
import torch

import oracle
import paper_1704_08907_amd as A

# float32 results against the float64 oracle: per element against the row's
# absolute-sum scale S_i of its summands (plus, for the neighbour sums, the
# rounding allowance of the oracle's RowScale), and normwise.
TOL_F32 = 1e-5
# float64: rounding of ~100-term sums with rsqrt/exp at ~1 ulp each
TOL_F64 = 1e-12


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def box_of(system, ncell=None):
    return A.BoxSpec(system.d, system.lo, system.hi, system.periodic, system.cutoff, ncell)


def torch_dtype(prec):
    return torch.float32 if prec == "f32" else torch.float64


def row_bound(scale, tol):
    """Per-row error bound: tol * S_i for a plain scale array (the dense sums),
    or the oracle's RowScale bound tol * S_i + 16 u_P D_i (the neighbour sums)."""
    if isinstance(scale, oracle.RowScale):
        return scale.bound(tol)
    return tol * np.asarray(scale, dtype=np.float64)


def check_close(got, ref, scale, tol, what="", normwise=True):
    """Per-element |got - ref|_inf <= row_bound(scale, tol), and normwise
    ||got - ref||_2 <= tol ||ref||_2 (over all rows, or over the rows that
    normwise selects when it is a slice or an index array).

    S_i is the sum of the magnitudes of row i's summands: the bound a sum's
    rounding error scales with; the neighbour sums add the rounding of each
    summand's displacement and distance (oracle RowScale).  The normwise test
    relative to ||ref|| is only meaningful when the rows do not cancel by
    orders of magnitude, so inputs built to cluster points within a few ulps
    of each other skip it.  Returns the largest per-row ratio error / bound."""
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    err = np.abs(got - ref).max(axis=1)
    bound = np.maximum(row_bound(scale, tol), 1e-300)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, "%s: %d elements over tolerance, worst row %d: got %s ref %s bound %g" % (
        what, bad.size, bad[0], got[bad[0]], ref[bad[0]], bound[bad[0]])
    sel = slice(None) if normwise is True else (None if normwise is False or normwise is None else normwise)
    if sel is not None:
        nref = np.linalg.norm(ref[sel])
        if nref > 0:
            nerr = np.linalg.norm(got[sel] - ref[sel])
            assert nerr <= tol * nref, "%s: normwise error %g" % (what, nerr / nref)
    return float((err / bound).max()) if err.size else 0.0


def download_u32(ptr, count):
    """Copy count uint32 values from a raw device pointer to a numpy array."""
    import ctypes as C
    out = np.zeros(max(count, 1), dtype=np.uint32)
    if count == 0:
        return out[:0]
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    torch.cuda.synchronize()
    st = hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), count * 4, 2)  # DeviceToHost
    assert st == 0
    return out[:count]


def download_f(ptr, count, dtype):
    import ctypes as C
    out = np.zeros(max(count, 1), dtype=dtype)
    if count == 0:
        return out[:0]
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    torch.cuda.synchronize()
    st = hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), count * out.itemsize, 2)
    assert st == 0
    return out[:count]


def cells_state(cells):
    """(keys, perm, offsets, x_sorted) of a GPU cell list as numpy arrays."""
    v = cells.view()
    n = int(v.n)
    keys = download_u32(v.keys, n)
    perm = download_u32(v.perm, n)
    off = download_u32(v.cell_offsets, int(v.ncells) + 1)
    dt = np.float32 if v.dtype == 0 else np.float64
    xs = download_f(v.x_sorted, n * int(v.x_pitch), dt).reshape(n, int(v.x_pitch))
    return keys, perm, off, xs


def oracle_pairs_sorted(g, x):
    return oracle.pairs(g, x, oracle.ROUTE_CELLS)


def gpu_pairs_sorted(ctx, cells):
    pi, pj = A.pair_list(ctx, cells)
    p = np.stack([pi.cpu().numpy().astype(np.uint32), pj.cpu().numpy().astype(np.uint32)], axis=1)
    if p.shape[0] == 0:
        return p.reshape(0, 2)
    return p[np.lexsort((p[:, 1], p[:, 0]))]
