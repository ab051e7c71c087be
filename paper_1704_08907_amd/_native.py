"""ctypes binding of libaboria_mi355x.so: argument marshalling only.

Every function here has the name of the C entry point it calls (without the
``aboria_`` prefix) and does no arithmetic of its own: device arrays are torch
tensors whose data pointers are handed over, and every step of the path runs in
the HIP kernels.  There is no CPU fallback: if the library is missing, loading
fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Union

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaboria_mi355x.so")

F32, F64 = 0, 1
OPS = {"count": 0, "spring": 1, "soft_sphere": 2, "exp_force": 3, "dem_spring": 4}
KERNELS = {"gaussian": 0, "multiquadric": 1}
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "DOMAIN", 3: "UNSUPPORTED", 4: "OUT_OF_MEMORY", 5: "DEVICE"}


class AboriaError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__("%s: %s (%s)" % (what, STATUS.get(code, code), msg))
        self.code = code
        self.status = STATUS.get(code, str(code))


class Box(C.Structure):
    _fields_ = [("d", C.c_int32), ("periodic", C.c_int32 * 3), ("ncell", C.c_int32 * 3),
                ("reach", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("cutoff", C.c_double)]


class CellsView(C.Structure):
    _fields_ = [("nsys", C.c_int32), ("d", C.c_int32), ("dtype", C.c_int32), ("sort_ipt", C.c_int32),
                ("n", C.c_int64), ("ncells", C.c_int64), ("perm", C.c_void_p), ("keys", C.c_void_p),
                ("cell_offsets", C.c_void_p), ("x_sorted", C.c_void_p), ("x_pitch", C.c_int32),
                ("bucket_bits", C.c_int32), ("ncell_host", C.POINTER(C.c_int32)),
                ("cell_base_host", C.POINTER(C.c_uint32)), ("sys_offsets_host", C.POINTER(C.c_int64))]


_lib = None
EXPORTS = ["aboria_create", "aboria_destroy", "aboria_set_stream", "aboria_last_error", "aboria_sync",
           "aboria_build_cells", "aboria_cells_view_get", "aboria_cells_destroy", "aboria_pair_sum",
           "aboria_pair_sum_backward", "aboria_pair_list", "aboria_dense_sum",
           "aboria_graph_capture_begin", "aboria_graph_capture_end", "aboria_graph_launch",
           "aboria_graph_destroy", "aboria_autotune", "aboria_variant_count", "aboria_variant_name",
           "aboria_set_variant", "aboria_op_ny", "aboria_op_na", "aboria_set_build_strategy",
           "aboria_build_neighbours", "aboria_neighbour_capacity", "aboria_integrate",
           "aboria_dense_sum_backward", "aboria_autotune_cells", "aboria_pair_sum_and_backward",
           "aboria_dense_sum_noalloc", "aboria_md_step", "aboria_cells_reorder", "aboria_selected_variant",
           "aboria_autotune_dense", "aboria_dense_plan_name", "aboria_set_dense_plan", "aboria_set_build_shape",
           "aboria_autotune_build"]


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run __graft_entry__.build() first" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        I32, I64 = C.c_int32, C.c_int64
        sig = {
            "aboria_create": ([I32, P, C.POINTER(P)], I32),
            "aboria_destroy": ([P], I32),
            "aboria_set_stream": ([P, P], I32),
            "aboria_last_error": ([P], C.c_char_p),
            "aboria_sync": ([P], I32),
            "aboria_build_cells": ([P, I32, I32, C.POINTER(Box), C.POINTER(I64), P, C.POINTER(P)], I32),
            "aboria_cells_view_get": ([P, C.POINTER(CellsView)], I32),
            "aboria_cells_destroy": ([P], I32),
            "aboria_pair_sum": ([P, P, I32, C.POINTER(C.c_double), I32, P, I32, P, I32], I32),
            "aboria_pair_sum_backward": ([P, P, I32, C.POINTER(C.c_double), I32, P, I32, P, I32, P, P], I32),
            "aboria_pair_list": ([P, P, I64, P, P, C.POINTER(I64)], I32),
            "aboria_dense_sum": ([P, I32, I32, C.POINTER(C.c_double), I32, I32, I64, P, I64, P, P, P], I32),
            "aboria_selected_variant": ([P, P, I32, I32, C.POINTER(I32)], I32),
            "aboria_autotune_dense": ([P, I32, I32, C.POINTER(C.c_double), I32, I32, I64, P, I64, P, P, P, P,
                                       C.POINTER(I32)], I32),
            "aboria_dense_plan_name": ([I32], C.c_char_p),
            "aboria_set_dense_plan": ([P, I32], I32),
            "aboria_set_build_shape": ([P, I32, I32, I32], I32),
            "aboria_autotune_build": ([P, I32, I32, P, C.POINTER(I64), P, C.POINTER(I32), C.POINTER(I32),
                                       C.POINTER(I32)], I32),
            "aboria_md_step": ([P, P, I32, C.POINTER(C.c_double), I32, C.c_double, P, P, P, P], I32),
            "aboria_cells_reorder": ([P, P, I32, C.POINTER(P), C.POINTER(I32)], I32),
            "aboria_dense_sum_noalloc": ([P, I32, I32, C.POINTER(C.c_double), I32, I32, I64, P, I64, P, P, P], I32),
            "aboria_graph_capture_begin": ([P], I32),
            "aboria_graph_capture_end": ([P, C.POINTER(P)], I32),
            "aboria_graph_launch": ([P, P], I32),
            "aboria_graph_destroy": ([P], I32),
            "aboria_autotune": ([P, P, I32, C.POINTER(C.c_double), I32, P, I32, P, I32, P, C.POINTER(I32)], I32),
            "aboria_variant_count": ([], I32),
            "aboria_variant_name": ([I32], C.c_char_p),
            "aboria_set_variant": ([P, I32], I32),
            "aboria_op_ny": ([I32, I32], I32),
            "aboria_op_na": ([I32], I32),
            "aboria_set_build_strategy": ([P, I32], I32),
            "aboria_build_neighbours": ([P, P, I32], I32),
            "aboria_neighbour_capacity": ([P], I32),
            "aboria_integrate": ([P, P, C.c_double, P, P, P], I32),
            "aboria_pair_sum_and_backward": ([P, P, I32, C.POINTER(C.c_double), I32, P, I32, P, I32, P, P, P],
                                             I32),
            "aboria_autotune_cells": ([P, I32, I32, C.POINTER(Box), C.POINTER(I64), P, I32, C.POINTER(C.c_double),
                                       I32, P, I32, P, I32, C.POINTER(Box), C.POINTER(C.c_double)], I32),
            "aboria_dense_sum_backward": ([P, I32, I32, C.POINTER(C.c_double), I32, I32, I64, P, I64, P, P, P,
                                           P, P, P], I32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("positions must be float32 or float64, got %s" % t.dtype)


def _check_dev(t: torch.Tensor, name: str, dtype=None):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))


class Context:
    """An aboria_ctx bound to one device and one stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib().aboria_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise AboriaError(st, "create", "device %d" % device)
        self.handle = h
        self.forced_variant = -1

    def check(self, st: int, what: str):
        if st != 0:
            raise AboriaError(st, what, self.last_error())

    def last_error(self) -> str:
        m = lib().aboria_last_error(self.handle)
        return m.decode() if m else ""

    def sync(self):
        self.check(lib().aboria_sync(self.handle), "sync")

    def set_stream(self, stream: torch.cuda.Stream):
        self.check(lib().aboria_set_stream(self.handle, C.c_void_p(stream.cuda_stream)), "set_stream")
        self.stream = stream

    def set_build_strategy(self, strategy: str):
        """Sort used by later builds: "radix" or "counting" (the same cell list either way)."""
        code = {"radix": 0, "counting": 1}[strategy]
        self.check(lib().aboria_set_build_strategy(self.handle, code), "set_build_strategy")

    def set_variant(self, v: int):
        """Force a neighbour-sum variant for later calls (-1 = tuned / default)."""
        self.check(lib().aboria_set_variant(self.handle, v), "set_variant")
        self.forced_variant = int(v)

    def set_dense_plan(self, plan: int):
        """Force a dense-sum launch plan for later calls (-1 = tuned / default)."""
        self.check(lib().aboria_set_dense_plan(self.handle, int(plan)), "set_dense_plan")

    def set_build_shape(self, ipt: int = 0, low_bits: int = 0, shuffle: int = 0):
        """Radix build shape for cell lists created later (0 = rule / tuned; shuffle 1 = on
        where it fits, 2 = off)."""
        self.check(lib().aboria_set_build_shape(self.handle, int(ipt), int(low_bits), int(shuffle)),
                   "set_build_shape")

    def close(self):
        if getattr(self, "handle", None):
            lib().aboria_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class BoxSpec:
    d: int
    lo: Sequence[float]
    hi: Sequence[float]
    periodic: Sequence[int]
    cutoff: float
    ncell: Optional[Sequence[int]] = None
    # cells searched on each side of a particle's cell (0 = 1): one value for every
    # dimension or one per dimension
    reach: Union[int, Sequence[int]] = 0

    def reach_list(self) -> list:
        r = [int(v) for v in self.reach] if hasattr(self.reach, "__len__") else [int(self.reach)] * self.d
        if len(r) != self.d:
            raise ValueError("reach needs one value or d values")
        return r

    def to_c(self) -> Box:
        b = Box()
        b.d = self.d
        for k, m in enumerate(self.reach_list()[:3]):  # the library rejects d > 3
            b.reach[k] = m
        for k in range(min(self.d, 3)):
            b.lo[k] = float(self.lo[k])
            b.hi[k] = float(self.hi[k])
            b.periodic[k] = int(bool(self.periodic[k]))
            b.ncell[k] = int(self.ncell[k]) if self.ncell is not None else 0
        b.cutoff = float(self.cutoff)
        return b


@dataclass
class Cells:
    ctx: Context
    handle: C.c_void_p
    n: int
    d: int
    dtype: torch.dtype
    nsys: int
    boxes: list = field(default_factory=list)
    offsets: list = field(default_factory=list)
    # host-side count of the builds into this cell list (1 after it is created):
    # a caller that keeps results tied to one build (an autograd graph) checks it
    builds: int = 1

    def view(self) -> CellsView:
        v = CellsView()
        st = lib().aboria_cells_view_get(self.handle, C.byref(v))
        if st != 0:
            raise AboriaError(st, "cells_view_get", "")
        return v

    def close(self):
        if getattr(self, "handle", None):
            lib().aboria_cells_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_cells(ctx: Context, x: torch.Tensor, boxes: Sequence[BoxSpec], offsets: Optional[Sequence[int]] = None,
                cells: Optional[Cells] = None) -> Cells:
    """aboria_build_cells: x[n][d] (float32/float64, device); boxes per system."""
    _check_dev(x, "x")
    boxes = list(boxes)
    nsys = len(boxes)
    n = int(x.shape[0])
    if offsets is None:
        if nsys != 1:
            raise ValueError("offsets are required for more than one system")
        offsets = [0, n]
    arr_b = (Box * nsys)(*[b.to_c() for b in boxes])
    arr_o = (C.c_int64 * (nsys + 1))(*[int(o) for o in offsets])
    h = C.c_void_p(cells.handle.value) if cells is not None else C.c_void_p()
    st = lib().aboria_build_cells(ctx.handle, _dtype_code(x), nsys, arr_b, arr_o, _ptr(x), C.byref(h))
    ctx.check(st, "build_cells")
    if cells is not None:
        cells.boxes, cells.offsets = boxes, list(offsets)
        cells.builds += 1
        return cells
    return Cells(ctx, h, n, boxes[0].d, x.dtype, nsys, boxes, list(offsets))


def autotune_build(ctx: Context, x: torch.Tensor, boxes: Sequence[BoxSpec],
                   offsets: Optional[Sequence[int]] = None) -> tuple:
    """aboria_autotune_build: times the radix build shapes for these boxes and caches the
    fastest; returns (keys per thread, bucket bits, shuffle)."""
    _check_dev(x, "x")
    boxes = list(boxes)
    nsys = len(boxes)
    if offsets is None:
        if nsys != 1:
            raise ValueError("offsets are required for more than one system")
        offsets = [0, int(x.shape[0])]
    arr_b = (Box * nsys)(*[b.to_c() for b in boxes])
    arr_o = (C.c_int64 * (nsys + 1))(*[int(o) for o in offsets])
    ipt, lb, sh = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    ctx.check(lib().aboria_autotune_build(ctx.handle, _dtype_code(x), nsys, arr_b, arr_o, _ptr(x), C.byref(ipt),
                                          C.byref(lb), C.byref(sh)), "autotune_build")
    return int(ipt.value), int(lb.value), int(sh.value)


def op_ny(op: str, d: int) -> int:
    return int(lib().aboria_op_ny(OPS[op], d))


def op_na(op: str) -> int:
    return int(lib().aboria_op_na(OPS[op]))


def _params(params):
    params = [float(p) for p in params]
    arr = (C.c_double * max(1, len(params)))(*params)
    return arr, len(params)


def pair_sum(ctx: Context, cells: Cells, op: str, params=(), a: Optional[torch.Tensor] = None,
             y: Optional[torch.Tensor] = None) -> torch.Tensor:
    """aboria_pair_sum: returns y[n][ny] in original particle order."""
    ny, na = op_ny(op, cells.d), op_na(op)
    if y is None:
        y = torch.empty((cells.n, ny), dtype=cells.dtype, device="cuda:%d" % ctx.device)
    _check_dev(y, "y", cells.dtype)
    if a is not None:
        _check_dev(a, "a", cells.dtype)
    arr, npar = _params(params)
    st = lib().aboria_pair_sum(ctx.handle, cells.handle, OPS[op], arr, npar, _ptr(a), na, _ptr(y), ny)
    ctx.check(st, "pair_sum")
    return y


def pair_sum_backward(ctx: Context, cells: Cells, op: str, params, gy: torch.Tensor,
                      a: Optional[torch.Tensor] = None, gx: Optional[torch.Tensor] = None,
                      ga: Optional[torch.Tensor] = None, want_ga: bool = True):
    """aboria_pair_sum_backward: returns (gx[n][d], ga[n][na] or None)."""
    ny, na = op_ny(op, cells.d), op_na(op)
    dev = "cuda:%d" % ctx.device
    _check_dev(gy, "gy", cells.dtype)
    if gx is None:
        gx = torch.empty((cells.n, cells.d), dtype=cells.dtype, device=dev)
    if ga is None and na > 0 and want_ga:
        ga = torch.empty((cells.n, na), dtype=cells.dtype, device=dev)
    arr, npar = _params(params)
    st = lib().aboria_pair_sum_backward(ctx.handle, cells.handle, OPS[op], arr, npar, _ptr(a), na, _ptr(gy), ny,
                                        _ptr(gx), _ptr(ga))
    ctx.check(st, "pair_sum_backward")
    return gx, ga


def pair_sum_and_backward(ctx: Context, cells: Cells, op: str, params, gy: torch.Tensor,
                          a: Optional[torch.Tensor] = None, y: Optional[torch.Tensor] = None,
                          gx: Optional[torch.Tensor] = None, want_ga: bool = True):
    """aboria_pair_sum_and_backward: (y, gx, ga) from one box search, gy known in advance."""
    ny, na = op_ny(op, cells.d), op_na(op)
    dev = "cuda:%d" % ctx.device
    _check_dev(gy, "gy", cells.dtype)
    if y is None:
        y = torch.empty((cells.n, ny), dtype=cells.dtype, device=dev)
    if gx is None:
        gx = torch.empty((cells.n, cells.d), dtype=cells.dtype, device=dev)
    ga = torch.empty((cells.n, na), dtype=cells.dtype, device=dev) if (na > 0 and want_ga) else None
    arr, npar = _params(params)
    st = lib().aboria_pair_sum_and_backward(ctx.handle, cells.handle, OPS[op], arr, npar, _ptr(a), na, _ptr(gy), ny,
                                            _ptr(y), _ptr(gx), _ptr(ga))
    ctx.check(st, "pair_sum_and_backward")
    return y, gx, ga


def build_neighbours(ctx: Context, cells: Cells, capacity: int = 0) -> int:
    """aboria_build_neighbours: records each particle's neighbour set on the
    cell list (later sums and adjoints on it replay the list); returns the
    entries kept per particle."""
    ctx.check(lib().aboria_build_neighbours(ctx.handle, cells.handle, int(capacity)), "build_neighbours")
    return int(lib().aboria_neighbour_capacity(cells.handle))


def integrate(ctx: Context, cells: Cells, dt: float, f: torch.Tensor, x: torch.Tensor, v: torch.Tensor):
    """aboria_integrate: v += dt f, then x += dt v, wrapped into the periodic box (in place)."""
    for t, name in ((f, "f"), (x, "x"), (v, "v")):
        _check_dev(t, name, cells.dtype)
        if tuple(t.shape) != (cells.n, cells.d):
            raise ValueError("%s must be [n][d]" % name)
    ctx.check(lib().aboria_integrate(ctx.handle, cells.handle, float(dt), _ptr(f), _ptr(x), _ptr(v)), "integrate")
    return x, v


def selected_variant(ctx: Context, cells: Cells, op: str, backward: bool = False) -> int:
    """aboria_selected_variant: the variant a sum (or adjoint) on cells would use now."""
    out = C.c_int32()
    ctx.check(lib().aboria_selected_variant(ctx.handle, cells.handle, OPS[op], int(bool(backward)), C.byref(out)),
              "selected_variant")
    return int(out.value)


def md_step(ctx: Context, cells: Cells, op: str, params, dt: float, x: Optional[torch.Tensor], v: torch.Tensor,
            x_out: Optional[torch.Tensor] = None, v_out: Optional[torch.Tensor] = None):
    """aboria_md_step: the force of op (exp_force or spring) by the box search and the
    Euler update in one kernel: in place on x and v, or, with x_out and v_out, written
    in cell order to them (x is then not read and may be None)."""
    for t, name in ((x, "x"), (v, "v"), (x_out, "x_out"), (v_out, "v_out")):
        if t is None:
            continue
        _check_dev(t, name, cells.dtype)
        if tuple(t.shape) != (cells.n, cells.d):
            raise ValueError("%s must be [n][d]" % name)
    arr, npar = _params(params)
    st = lib().aboria_md_step(ctx.handle, cells.handle, OPS[op], arr, npar, float(dt), _ptr(x), _ptr(v),
                              _ptr(x_out), _ptr(v_out))
    ctx.check(st, "md_step")
    return (x, v) if x_out is None else (x_out, v_out)


def cells_reorder(ctx: Context, cells: Cells, *bufs: torch.Tensor):
    """aboria_cells_reorder: permutes each [n][...] device tensor into the cell order in
    place and makes that the cell list's particle order."""
    for t in bufs:
        if t.device.type != "cuda" or not t.is_contiguous() or int(t.shape[0]) != cells.n:
            raise ValueError("reorder buffers must be contiguous [n][...] device tensors")
    ptrs = (C.c_void_p * max(1, len(bufs)))(*[t.data_ptr() for t in bufs])
    sizes = (C.c_int32 * max(1, len(bufs)))(*[t.element_size() * (t.numel() // max(1, cells.n)) for t in bufs])
    ctx.check(lib().aboria_cells_reorder(ctx.handle, cells.handle, len(bufs), ptrs, sizes), "cells_reorder")
    return bufs


def pair_list(ctx: Context, cells: Cells):
    """aboria_pair_list: (pi, pj) uint32->int64 device tensors of all ordered pairs."""
    total = C.c_int64()
    st = lib().aboria_pair_list(ctx.handle, cells.handle, 0, None, None, C.byref(total))
    ctx.check(st, "pair_list")
    m = int(total.value)
    dev = "cuda:%d" % ctx.device
    pi = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    pj = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    st = lib().aboria_pair_list(ctx.handle, cells.handle, m, _ptr(pi), _ptr(pj), C.byref(total))
    ctx.check(st, "pair_list")
    return pi[:m], pj[:m]


def dense_sum(ctx: Context, xt: torch.Tensor, xs: torch.Tensor, w: torch.Tensor, sigma: float,
              y: Optional[torch.Tensor] = None, kernel: str = "gaussian") -> torch.Tensor:
    """aboria_dense_sum: y[i] = sum_j K(xt_i, xs_j) w_j (sigma is the kernel's parameter:
    the Gaussian's width or the multiquadric's c)."""
    _check_dev(xt, "xt")
    _check_dev(xs, "xs", xt.dtype)
    _check_dev(w, "w", xt.dtype)
    d = int(xt.shape[1])
    if y is None:
        y = torch.empty(int(xt.shape[0]), dtype=xt.dtype, device=xt.device)
    _check_dev(y, "y", xt.dtype)
    arr, npar = _params([sigma])
    st = lib().aboria_dense_sum(ctx.handle, _dtype_code(xt), KERNELS[kernel], arr, npar, d, int(xt.shape[0]),
                                _ptr(xt), int(xs.shape[0]), _ptr(xs), _ptr(w), _ptr(y))
    ctx.check(st, "dense_sum")
    return y


def autotune_dense(ctx: Context, xt: torch.Tensor, xs: torch.Tensor, w: torch.Tensor, sigma: float,
                   gy: Optional[torch.Tensor] = None, kernel: str = "gaussian") -> int:
    """aboria_autotune_dense: times the dense launch plans of the forward (gy None) or the
    backward and caches the fastest; returns the chosen plan."""
    _check_dev(xt, "xt")
    _check_dev(xs, "xs", xt.dtype)
    _check_dev(w, "w", xt.dtype)
    d, nt, ns = int(xt.shape[1]), int(xt.shape[0]), int(xs.shape[0])
    if gy is not None:
        _check_dev(gy, "gy", xt.dtype)
        scratch = torch.empty(d * nt + (d + 1) * ns, dtype=xt.dtype, device=xt.device)
    else:
        scratch = torch.empty(nt, dtype=xt.dtype, device=xt.device)
    arr, npar = _params([sigma])
    out = C.c_int32(-1)
    st = lib().aboria_autotune_dense(ctx.handle, _dtype_code(xt), KERNELS[kernel], arr, npar, d, nt, _ptr(xt), ns,
                                     _ptr(xs), _ptr(w), _ptr(gy) if gy is not None else None, _ptr(scratch),
                                     C.byref(out))
    ctx.check(st, "autotune_dense")
    return int(out.value)


def dense_plan_name(plan: int) -> str:
    return lib().aboria_dense_plan_name(int(plan)).decode()


def dense_sum_noalloc(ctx: Context, xt: torch.Tensor, xs: torch.Tensor, w: torch.Tensor, sigma: float,
                      y: torch.Tensor, kernel: str = "gaussian") -> torch.Tensor:
    """aboria_dense_sum_noalloc: dense_sum into a caller-given y, with the library's
    fixed per-device scratch (no device allocation by the library)."""
    _check_dev(xt, "xt")
    _check_dev(xs, "xs", xt.dtype)
    _check_dev(w, "w", xt.dtype)
    _check_dev(y, "y", xt.dtype)
    arr, npar = _params([sigma])
    st = lib().aboria_dense_sum_noalloc(ctx.handle, _dtype_code(xt), KERNELS[kernel], arr, npar, int(xt.shape[1]),
                                        int(xt.shape[0]), _ptr(xt), int(xs.shape[0]), _ptr(xs), _ptr(w), _ptr(y))
    ctx.check(st, "dense_sum_noalloc")
    return y


def dense_sum_backward(ctx: Context, xt: torch.Tensor, xs: torch.Tensor, w: torch.Tensor, sigma: float,
                       gy: torch.Tensor, kernel: str = "gaussian", want=("xt", "xs", "w")):
    """aboria_dense_sum_backward: (gxt, gxs, gw) for L = sum_i gy_i y_i (None where not wanted)."""
    for t, name in ((xt, "xt"), (xs, "xs"), (w, "w"), (gy, "gy")):
        _check_dev(t, name, xt.dtype)
    d, nt, ns = int(xt.shape[1]), int(xt.shape[0]), int(xs.shape[0])
    gxt = torch.empty((nt, d), dtype=xt.dtype, device=xt.device) if "xt" in want else None
    gxs = torch.empty((ns, d), dtype=xt.dtype, device=xt.device) if "xs" in want else None
    gw = torch.empty(ns, dtype=xt.dtype, device=xt.device) if "w" in want else None
    arr, npar = _params([sigma])
    st = lib().aboria_dense_sum_backward(ctx.handle, _dtype_code(xt), KERNELS[kernel], arr, npar, d, nt, _ptr(xt),
                                         ns, _ptr(xs), _ptr(w), _ptr(gy), _ptr(gxt), _ptr(gxs), _ptr(gw))
    ctx.check(st, "dense_sum_backward")
    return gxt, gxs, gw


class Graph:
    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if getattr(self, "handle", None):
            lib().aboria_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_capture_begin(ctx: Context):
    ctx.check(lib().aboria_graph_capture_begin(ctx.handle), "graph_capture_begin")


def graph_capture_end(ctx: Context) -> Graph:
    h = C.c_void_p()
    ctx.check(lib().aboria_graph_capture_end(ctx.handle, C.byref(h)), "graph_capture_end")
    return Graph(h)


def graph_launch(ctx: Context, g: Graph):
    ctx.check(lib().aboria_graph_launch(ctx.handle, g.handle), "graph_launch")


def autotune(ctx: Context, cells: Cells, op: str, params=(), a: Optional[torch.Tensor] = None,
             gy: Optional[torch.Tensor] = None) -> int:
    """aboria_autotune: tunes the forward sum (gy None) or the adjoint for gy; returns the variant."""
    ny, na = op_ny(op, cells.d), op_na(op)
    width = ny if gy is None else cells.d
    out = torch.empty((cells.n, width), dtype=cells.dtype, device="cuda:%d" % ctx.device)
    if gy is not None:
        _check_dev(gy, "gy", cells.dtype)
    arr, npar = _params(params)
    choice = C.c_int32(-1)
    st = lib().aboria_autotune(ctx.handle, cells.handle, OPS[op], arr, npar, _ptr(a), na, _ptr(gy), ny, _ptr(out),
                               C.byref(choice))
    ctx.check(st, "autotune")
    return int(choice.value)


def autotune_cells(ctx: Context, x: torch.Tensor, boxes: Sequence[BoxSpec], offsets: Optional[Sequence[int]],
                   op: str, params=(), a: Optional[torch.Tensor] = None, gy: Optional[torch.Tensor] = None):
    """aboria_autotune_cells: (boxes with the fastest explicit cell counts, the chosen scale factor)."""
    _check_dev(x, "x")
    boxes = list(boxes)
    nsys = len(boxes)
    if offsets is None:
        offsets = [0, int(x.shape[0])]
    d = boxes[0].d
    arr_b = (Box * nsys)(*[b.to_c() for b in boxes])
    out_b = (Box * nsys)()
    arr_o = (C.c_int64 * (nsys + 1))(*[int(o) for o in offsets])
    arr, npar = _params(params)
    factor = C.c_double(0.0)
    st = lib().aboria_autotune_cells(ctx.handle, _dtype_code(x), nsys, arr_b, arr_o, _ptr(x), OPS[op], arr, npar,
                                     _ptr(a), op_na(op), _ptr(gy), op_ny(op, d), out_b, C.byref(factor))
    ctx.check(st, "autotune_cells")
    tuned = [BoxSpec(b.d, b.lo, b.hi, b.periodic, b.cutoff, [int(out_b[i].ncell[k]) for k in range(d)],
                     [int(out_b[i].reach[k]) for k in range(d)]) for i, b in enumerate(boxes)]
    return tuned, float(factor.value)


def variant_count() -> int:
    return int(lib().aboria_variant_count())


def variant_name(v: int) -> str:
    return lib().aboria_variant_name(v).decode()
