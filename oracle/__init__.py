"""CPU oracle for the cell-list neighbour operators and the dense kernel sum.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path (the HIP library and its
Python binding) never imports this package, and this package imports nothing
from the product.  The arithmetic lives in ``oracle.c`` (plain C, float64 sums,
input-precision pair predicate); this module only compiles it with gcc and
marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

F32, F64 = 0, 1
OPS = {"count": 0, "spring": 1, "soft_sphere": 2, "exp_force": 3, "dem_spring": 4}
ROUTE_BRUTE, ROUTE_CELLS = 0, 1
OK, ERR_INVALID, ERR_DOMAIN, ERR_UNSUPPORTED, ERR_NOMEM = 0, 1, 2, 3, 4


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with oracle status %d" % (what, code))
        self.code = code


def build() -> str:
    """Compile oracle.c.  Contraction is off so that every fma is the explicit one."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", LIB + ".tmp", SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Grid(C.Structure):
    _fields_ = [("d", C.c_int32), ("dtype", C.c_int32), ("periodic", C.c_int32 * 3),
                ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("L", C.c_double * 3), ("inv_w", C.c_double * 3), ("r", C.c_double),
                ("r2", C.c_double), ("ncells", C.c_int64), ("reach", C.c_int32 * 3), ("pad", C.c_int32)]

    @property
    def ncell(self):
        return [self.n[k] for k in range(self.d)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.or_grid_init.argtypes = [C.POINTER(Grid), C.c_int32, C.c_int32, P, P, P, C.c_double, P, P]
        L.or_cell_ids.argtypes = [C.POINTER(Grid), C.c_int64, P, P]
        L.or_sort_cells.argtypes = [C.POINTER(Grid), C.c_int64, P, P, P]
        L.or_pairs.argtypes = [C.POINTER(Grid), C.c_int32, C.c_int64, P, C.c_int64, P, P]
        L.or_pairs.restype = C.c_int64
        L.or_pair_sum.argtypes = [C.POINTER(Grid), C.c_int32, C.c_int32, P, C.c_int64, P, P,
                                  C.c_int64, P, P, P, P, C.c_int32]
        L.or_pair_sum_backward.argtypes = [C.POINTER(Grid), C.c_int32, C.c_int32, P, C.c_int64, P, P,
                                           P, C.c_int64, P, P, P, P, P, P, P, C.c_int32]
        L.or_fd_grad.argtypes = [C.POINTER(Grid), C.c_int32, P, C.c_int64, P, P, P, C.c_int64, P,
                                 C.c_double, P]
        L.or_dense_gauss.argtypes = [C.c_int32, C.c_int64, P, C.c_int64, P, P, C.c_double,
                                     C.c_int64, P, P, P]
        L.or_md_step.argtypes = [C.POINTER(Grid), C.c_int32, C.c_double, C.c_double, C.c_int64, P, P, P, P]
        L.or_dense_sum.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_int64, P, C.c_int64, P, P, P, P]
        L.or_dense_backward.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_int64, P, C.c_int64, P, P, P,
                                        P, P, P, P, P, P]
        L.or_tie_band.argtypes = [C.POINTER(Grid), C.c_int64, P]
        L.or_tie_band.restype = C.c_int64
        L.or_op_ny.argtypes = [C.c_int32, C.c_int32]
        L.or_op_ny.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def grid(d, lo, hi, periodic, cutoff, precision="f64", ncell=None, reach=1) -> Grid:
    """The cell grid of a box (cell count rule R1 for search reach m = reach,
    one value for every dimension or one per dimension; P-rounded box, 1/w)."""
    g = Grid()
    lo_a = np.zeros(3); lo_a[:d] = lo
    hi_a = np.ones(3); hi_a[:d] = hi
    per = np.zeros(3, dtype=np.int32); per[:d] = periodic
    nreq = np.zeros(3, dtype=np.int32)
    if ncell is not None:
        nreq[:d] = ncell
    m = np.ones(3, dtype=np.int32)
    m[:d] = reach
    st = lib().or_grid_init(C.byref(g), d, F32 if precision == "f32" else F64, _ptr(lo_a),
                            _ptr(hi_a), _ptr(per), float(cutoff), _ptr(nreq), _ptr(m))
    if st != OK:
        raise OracleError(st, "grid")
    return g


def grid_of(system, ncell=None, reach=1) -> Grid:
    return grid(system.d, system.lo, system.hi, system.periodic, system.cutoff,
                system.precision, ncell, reach)


def cell_ids(g: Grid, x) -> tuple:
    """(ids, status): linear cell id per point; status OK or ERR_DOMAIN."""
    x = _f64(x)
    n = x.shape[0]
    ids = np.zeros(n, dtype=np.uint32)
    st = lib().or_cell_ids(C.byref(g), n, _ptr(x), _ptr(ids))
    return ids, st


def sort_cells(g: Grid, ids):
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n = ids.shape[0]
    perm = np.zeros(n, dtype=np.uint32)
    off = np.zeros(g.ncells + 1, dtype=np.uint32)
    st = lib().or_sort_cells(C.byref(g), n, _ptr(ids), _ptr(perm), _ptr(off))
    if st != OK:
        raise OracleError(st, "sort_cells")
    return perm, off


def pairs(g: Grid, x, route=ROUTE_CELLS):
    """All ordered pairs (i, j), sorted lexicographically, as an [m][2] uint32 array."""
    x = _f64(x)
    n = x.shape[0]
    m = lib().or_pairs(C.byref(g), route, n, _ptr(x), 0, None, None)
    if m < 0:
        raise OracleError(ERR_NOMEM, "pairs")
    pi = np.zeros(max(m, 1), dtype=np.uint32)
    pj = np.zeros(max(m, 1), dtype=np.uint32)
    m2 = lib().or_pairs(C.byref(g), route, n, _ptr(x), m, _ptr(pi), _ptr(pj))
    assert m2 == m
    p = np.stack([pi[:m], pj[:m]], axis=1)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return p[order]


def op_ny(op: str, d: int) -> int:
    return lib().or_op_ny(OPS[op], d)


# Allowance for the rounding of a summand's displacement and distance, in units
# of the working precision's unit roundoff (reading R6 in oracle.c).
COND_ULPS = 16.0


class RowScale:
    """The two per-row scales of reading R6 (oracle.c) for one output.

    s[row]: sum over the row's summands of their max-norm (the absolute-sum
    scale of a relative tolerance).  d[row]: sum over the row's summands of
    their condition with respect to the pair displacement.  u: unit roundoff
    of the working precision.  A result row passes at tolerance tol when
    |got - ref|_inf <= tol * s + COND_ULPS * u * d."""

    def __init__(self, s, d, u):
        self.s = np.asarray(s, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)
        self.u = float(u)

    def bound(self, tol):
        return tol * self.s + COND_ULPS * self.u * self.d

    def __getitem__(self, idx):
        return RowScale(self.s[idx], self.d[idx], self.u)

    def __len__(self):
        return self.s.shape[0]


def unit_roundoff(g: Grid) -> float:
    return 2.0 ** -24 if g.dtype == F32 else 2.0 ** -53


def _threads(nthreads):
    if nthreads is None:
        return 1
    if nthreads == "all":
        return len(os.sched_getaffinity(0))
    return max(1, int(nthreads))


def pair_sum(g: Grid, op: str, params, x, a=None, rows=None, route=ROUTE_CELLS, scales=True, nthreads=None):
    """(y, RowScale) in float64, or y alone with scales=False (then nothing
    beyond the plain sum is computed).  nthreads: threads over rows (an
    integer, or "all" for every core this process may run on)."""
    x = _f64(x)
    n = x.shape[0]
    a = _f64(a)
    prm = np.zeros(4); prm[:len(params)] = params
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if rows is None else rows_a.shape[0]
    ny = op_ny(op, g.d)
    y = np.zeros((m, ny))
    sc = np.zeros(m) if scales else None
    cd = np.zeros(m) if scales else None
    st = lib().or_pair_sum(C.byref(g), route, OPS[op], _ptr(prm), n, _ptr(x),
                           _ptr(a if a is None else a.reshape(-1)), m if rows is not None else 0,
                           _ptr(rows_a), _ptr(y), _ptr(sc), _ptr(cd), _threads(nthreads))
    if st != OK:
        raise OracleError(st, "pair_sum")
    return (y, RowScale(sc, cd, unit_roundoff(g))) if scales else y


KERNELS = {"gaussian": 0, "multiquadric": 1}


def dense_sum(kernel: str, prm: float, xt, xs, w):
    """(y, scale): y_i = sum_j K(xt_i, xs_j) w_j in float64 (Gaussian: prm = sigma;
    multiquadric sqrt(q + c^2): prm = c)."""
    xt, xs, w = _f64(xt), _f64(xs), _f64(w).reshape(-1)
    d = xt.shape[1]
    y = np.zeros(xt.shape[0])
    sc = np.zeros(xt.shape[0])
    st = lib().or_dense_sum(KERNELS[kernel], float(prm), d, xt.shape[0], _ptr(xt), xs.shape[0], _ptr(xs), _ptr(w),
                            _ptr(y), _ptr(sc))
    if st != OK:
        raise OracleError(st, "dense_sum")
    return y, sc


def dense_backward(kernel: str, prm: float, xt, xs, w, gy):
    """Adjoint of dense_sum for L = sum_i gy_i y_i, float64:
    (gxt, gxs, gw, scale_xt, scale_xs, scale_w)."""
    xt, xs, w, gy = _f64(xt), _f64(xs), _f64(w).reshape(-1), _f64(gy).reshape(-1)
    d = xt.shape[1]
    nt, ns = xt.shape[0], xs.shape[0]
    gxt, gxs, gw = np.zeros((nt, d)), np.zeros((ns, d)), np.zeros(ns)
    sxt, sxs, sgw = np.zeros(nt), np.zeros(ns), np.zeros(ns)
    st = lib().or_dense_backward(KERNELS[kernel], float(prm), d, nt, _ptr(xt), ns, _ptr(xs), _ptr(w), _ptr(gy),
                                 _ptr(gxt), _ptr(gxs), _ptr(gw), _ptr(sxt), _ptr(sxs), _ptr(sgw))
    if st != OK:
        raise OracleError(st, "dense_backward")
    return gxt, gxs, gw, sxt, sxs, sgw


def md_step(g: Grid, c: float, dt: float, x, v, route=ROUTE_CELLS):
    """One time step of the Section 3 example in float64: returns (x_new, v_new, scale_v).

    v_new = v + dt (c S), S_i = sum_j -exp(-|dx|) dx/|dx| over the neighbours;
    x_new = x + dt v_new wrapped into the box in periodic dimensions; scale_v
    is the RowScale of the velocity change dt c S."""
    x = np.array(_f64(x), dtype=np.float64, copy=True, order="C")
    v = np.array(_f64(v), dtype=np.float64, copy=True, order="C")
    n = x.shape[0]
    sc = np.zeros(max(n, 1))
    cd = np.zeros(max(n, 1))
    st = lib().or_md_step(C.byref(g), route, float(c), float(dt), n, _ptr(x), _ptr(v), _ptr(sc), _ptr(cd))
    if st != OK:
        raise OracleError(st, "md_step")
    return x, v, RowScale(sc[:n], cd[:n], unit_roundoff(g))


def pair_sum_backward(g: Grid, op: str, params, x, gy, a=None, rows=None, route=ROUTE_CELLS, scales=True,
                      nthreads=None):
    """(gx, ga, RowScale of gx, RowScale of ga) in float64 for L = sum_i gy_i . y_i,
    or (gx, ga) with scales=False.  nthreads as in pair_sum."""
    x = _f64(x)
    n = x.shape[0]
    a = _f64(a)
    gy = _f64(gy).reshape(n, -1)
    prm = np.zeros(4); prm[:len(params)] = params
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if rows is None else rows_a.shape[0]
    gx = np.zeros((m, g.d))
    ga = np.zeros(m)
    sx, cx, sa, ca = ((np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m)) if scales else (None,) * 4)
    st = lib().or_pair_sum_backward(C.byref(g), route, OPS[op], _ptr(prm), n, _ptr(x),
                                    _ptr(a if a is None else a.reshape(-1)), _ptr(gy),
                                    m if rows is not None else 0, _ptr(rows_a), _ptr(gx),
                                    _ptr(ga), _ptr(sx), _ptr(cx), _ptr(sa), _ptr(ca), _threads(nthreads))
    if st != OK:
        raise OracleError(st, "pair_sum_backward")
    if not scales:
        return gx, ga
    u = unit_roundoff(g)
    return gx, ga, RowScale(sx, cx, u), RowScale(sa, ca, u)


def fd_grad(g: Grid, op: str, params, x, gy, coords, h, a=None):
    """Local central finite differences of L = sum_i gy_i . y_i (pair set fixed at x)."""
    x = _f64(x)
    n = x.shape[0]
    a = _f64(a)
    gy = _f64(gy).reshape(n, -1)
    prm = np.zeros(4); prm[:len(params)] = params
    coords = np.ascontiguousarray(coords, dtype=np.int64)
    out = np.zeros(coords.shape[0])
    st = lib().or_fd_grad(C.byref(g), OPS[op], _ptr(prm), n, _ptr(x),
                          _ptr(a if a is None else a.reshape(-1)), _ptr(gy), coords.shape[0],
                          _ptr(coords), float(h), _ptr(out))
    if st != OK:
        raise OracleError(st, "fd_grad")
    return out


def dense_gauss(xt, xs, w, sigma, rows=None):
    """(y, scale): Gaussian kernel sum in float64 over all sources (j = i included)."""
    xt = _f64(xt)
    xs = _f64(xs)
    w = _f64(w).reshape(-1)
    d = xt.shape[1]
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = xt.shape[0] if rows is None else rows_a.shape[0]
    y = np.zeros(m)
    sc = np.zeros(m)
    st = lib().or_dense_gauss(d, xt.shape[0], _ptr(xt), xs.shape[0], _ptr(xs), _ptr(w), float(sigma),
                              m if rows is not None else 0, _ptr(rows_a), _ptr(y), _ptr(sc))
    if st != OK:
        raise OracleError(st, "dense_gauss")
    return y, sc


def tie_band(g: Grid, x) -> int:
    x = _f64(x)
    return int(lib().or_tie_band(C.byref(g), x.shape[0], _ptr(x)))
