"""ctypes binding of libgridpull.so (the C ABI in include/gridpull.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions carry the ABI's names; device arrays are passed as torch tensors
(their data pointers), and work is enqueued on torch's current stream.  If
the library has not been built, loading fails with an error instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgridpull.so")

GP_OK = 0
GP_ERR_CAPACITY = 3
STATUS = {0: "GP_OK", 1: "GP_ERR_ARG", 2: "GP_ERR_DOMAIN", 3: "GP_ERR_CAPACITY", 4: "GP_ERR_OOM",
          5: "GP_ERR_DEVICE", 6: "GP_ERR_STATE", 7: "GP_ERR_NUMERIC"}

EXPORTS = ("gp_create", "gp_destroy", "gp_last_error", "gp_set_stream", "gp_sync", "gp_build_band",
           "gp_nn_query", "gp_set_nn_params", "gp_get_nn_params", "gp_get_nn_grid", "gp_autotune_nn", "gp_set_tv_layout", "gp_set_grad_params", "gp_get_grad_params", "gp_autotune_grad", "gp_sample_queries", "gp_pull_forward", "gp_pull_forward_static", "gp_forward_token", "gp_pull_backward", "gp_pull_forward_backward", "gp_pull_normals", "gp_step",
           "gp_shape_slots", "gp_export_layout", "gp_export_active_cells", "gp_extract_surface", "gp_gather_vertices", "gp_scatter_vertices",
           "gp_init_sphere", "gp_timing_enable", "gp_timing_report")


class GridPullError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class gp_shape(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("point_off", ctypes.c_int64), ("point_cnt", ctypes.c_int64),
                ("query_off", ctypes.c_int64), ("query_cnt", ctypes.c_int64)]


class gp_weights(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("beta", ctypes.c_float), ("gamma", ctypes.c_float)]


class gp_nn_params(ctypes.Structure):
    _fields_ = [("group_span", ctypes.c_int32), ("first_shell", ctypes.c_int32), ("tile_parts", ctypes.c_int32),
                ("skip_empty", ctypes.c_int32), ("morton_sort", ctypes.c_int32), ("cell_points", ctypes.c_int32)]

    def as_tuple(self) -> Tuple[int, int, int, int, int, int]:
        return (self.group_span, self.first_shell, self.tile_parts, self.skip_empty, self.morton_sort,
                self.cell_points)


class gp_grad_params(ctypes.Structure):
    _fields_ = [("window_cap", ctypes.c_int32), ("window_max_passes", ctypes.c_int32),
                ("tv_forward_wave_from", ctypes.c_int64), ("tv_backward_wave_from", ctypes.c_int64)]

    def as_tuple(self) -> Tuple[int, int, int, int]:
        return (self.window_cap, self.window_max_passes, self.tv_forward_wave_from, self.tv_backward_wave_from)


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libgridpull.so is not built (%s); run `python -m paper_2308_13175_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, i32, i64, u64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
    st = ctypes.c_int
    sig = {
        "gp_create": (st, [ctypes.POINTER(P), ctypes.c_int, P]),
        "gp_destroy": (None, [P]),
        "gp_last_error": (ctypes.c_char_p, [P]),
        "gp_set_stream": (st, [P, P]),
        "gp_sync": (st, [P]),
        "gp_build_band": (st, [P, ctypes.POINTER(gp_shape), i32, P, P, P, i32, i32, i32,
                               ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "gp_nn_query": (st, [P, P, P, P, i64, P]),
        "gp_set_nn_params": (st, [P, ctypes.POINTER(gp_nn_params)]),
        "gp_set_tv_layout": (st, [P, i32]),
        "gp_set_grad_params": (st, [P, ctypes.POINTER(gp_grad_params)]),
        "gp_get_grad_params": (st, [P, ctypes.POINTER(gp_grad_params)]),
        "gp_autotune_grad": (st, [P, P, P, P, P, i64, P, gp_weights, i32, ctypes.POINTER(gp_grad_params), P]),
        "gp_get_nn_params": (st, [P, ctypes.POINTER(gp_nn_params)]),
        "gp_get_nn_grid": (st, [P, i32, P, P]),
        "gp_autotune_nn": (st, [P, P, P, P, i64, P, i32, ctypes.POINTER(gp_nn_params), ctypes.POINTER(f32)]),
        "gp_sample_queries": (st, [P, u64, i32, P, f32, P, P, P, P]),
        "gp_pull_forward": (st, [P, P, P, P, P, i64, P, gp_weights, P, P]),
        "gp_pull_backward": (st, [P, P, P, P, P, i64, P, gp_weights, P, P, u64]),
        "gp_forward_token": (u64, [P]),
        "gp_pull_forward_static": (st, [P, P, P, P, P, i64, P, gp_weights, P, P]),
        "gp_pull_forward_backward": (st, [P, P, P, P, P, i64, P, gp_weights, P, P, P, P]),
        "gp_pull_normals": (st, [P, P, P, P, P, i64, P, P, P, P, f32, P, P, P]),
        "gp_step": (st, [P, P, P, P, P, i32, f32, f32, i32, f32, f32, f32]),
        "gp_shape_slots": (st, [P, P]),
        "gp_export_layout": (st, [P, P, P]),
        "gp_export_active_cells": (st, [P, i32, P, i64, ctypes.POINTER(i64)]),
        "gp_extract_surface": (st, [P, i32, P, P, P, i64, ctypes.POINTER(i64), i32]),
        "gp_gather_vertices": (st, [P, P, P]),
        "gp_scatter_vertices": (st, [P, P, P]),
        "gp_init_sphere": (st, [P, P, P, P]),
        "gp_timing_enable": (st, [P, ctypes.c_int]),
        "gp_timing_report": (st, [P, ctypes.c_char_p, i64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor], dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, status: int):
    if status != GP_OK:
        msg = load_library().gp_last_error(ctx)
        raise GridPullError(status, msg.decode() if msg else "")


def _stream(ctx):
    _check(ctx, load_library().gp_set_stream(ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def make_shape(dims: Sequence[int], lo: Sequence[float], hi: Sequence[float], point_off: int, point_cnt: int,
               query_off: int, query_cnt: int) -> gp_shape:
    s = gp_shape()
    for a in range(3):
        s.dims[a] = int(dims[a])
        s.lo[a] = float(lo[a])
        s.hi[a] = float(hi[a])
    s.point_off, s.point_cnt = int(point_off), int(point_cnt)
    s.query_off, s.query_cnt = int(query_off), int(query_cnt)
    return s


# ---- the ABI, one function per entry point ---------------------------------

def gp_create(device: int = 0, stream: Optional[int] = None):
    lib = load_library()
    ctx = ctypes.c_void_p()
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    st = lib.gp_create(ctypes.byref(ctx), int(device), ctypes.c_void_p(stream))
    if st != GP_OK:
        raise GridPullError(st, "gp_create failed")
    return ctx


def gp_destroy(ctx) -> None:
    load_library().gp_destroy(ctx)


def gp_last_error(ctx) -> str:
    m = load_library().gp_last_error(ctx)
    return m.decode() if m else ""


def gp_set_stream(ctx, stream: int) -> None:
    _check(ctx, load_library().gp_set_stream(ctx, ctypes.c_void_p(stream)))


def gp_sync(ctx) -> None:
    _check(ctx, load_library().gp_sync(ctx))


def gp_build_band(ctx, shapes: Sequence[gp_shape], px, py, pz, m1: int, m2: int, brick: int = 8):
    lib = load_library()
    _stream(ctx)
    arr = (gp_shape * len(shapes))(*shapes)
    n_slots = ctypes.c_int64()
    n_act = ctypes.c_int64()
    _check(ctx, lib.gp_build_band(ctx, arr, len(shapes), _ptr(px, torch.float32), _ptr(py, torch.float32),
                                  _ptr(pz, torch.float32), int(m1), int(m2), int(brick),
                                  ctypes.byref(n_slots), ctypes.byref(n_act)))
    return n_slots.value, n_act.value


def gp_nn_query(ctx, qx, qy, qz, nn_out) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_nn_query(ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32),
                                           _ptr(qz, torch.float32), qx.numel(), _ptr(nn_out, torch.int32)))


def gp_set_nn_params(ctx, group_span: int, first_shell: int, tile_parts: int = 1, skip_empty: int = 0,
                     morton_sort: int = 1, cell_points: int = 8) -> None:
    """A new cell_points rebuilds the search grids of a built context."""
    p = gp_nn_params(int(group_span), int(first_shell), int(tile_parts), int(skip_empty), int(morton_sort),
                     int(cell_points))
    _check(ctx, load_library().gp_set_nn_params(ctx, ctypes.byref(p)))


def gp_get_nn_grid(ctx, shape: int) -> Tuple[Tuple[int, int, int], int]:
    """((cells per axis of the shape's search grid), k): its cells are 2^k band cells wide."""
    dims, level = (ctypes.c_int32 * 3)(), ctypes.c_int32(0)
    _check(ctx, load_library().gp_get_nn_grid(ctx, int(shape), dims, ctypes.byref(level)))
    return (dims[0], dims[1], dims[2]), level.value


def gp_set_tv_layout(ctx, layout: int) -> None:
    """0: by band size, 1: one block per brick, 2: one wave per brick."""
    _check(ctx, load_library().gp_set_tv_layout(ctx, int(layout)))


def gp_set_grad_params(ctx, window_cap: int = 4096, window_max_passes: int = 16,
                       tv_forward_wave_from: int = 2048, tv_backward_wave_from: int = 16384) -> None:
    p = gp_grad_params(int(window_cap), int(window_max_passes), int(tv_forward_wave_from),
                       int(tv_backward_wave_from))
    _check(ctx, load_library().gp_set_grad_params(ctx, ctypes.byref(p)))


def gp_get_grad_params(ctx) -> Tuple[int, int, int, int]:
    """(window_cap, window_max_passes, tv_forward_wave_from, tv_backward_wave_from)."""
    p = gp_grad_params()
    _check(ctx, load_library().gp_get_grad_params(ctx, ctypes.byref(p)))
    return p.as_tuple()


def gp_autotune_grad(ctx, qx, qy, qz, nn, field, weights, reps: int = 2):
    """Time the gradient-pass and TV settings on these inputs and keep the fastest:
    ((window_cap, window_max_passes, tv_forward_wave_from, tv_backward_wave_from),
     (query pass ms, TV forward ms, TV backward ms))."""
    _stream(ctx)
    p, ms = gp_grad_params(), (ctypes.c_float * 3)()
    _check(ctx, load_library().gp_autotune_grad(ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32),
                                                _ptr(qz, torch.float32), _ptr(nn, torch.int32), qx.numel(),
                                                _ptr(field, torch.float32), _weights(*weights), int(reps),
                                                ctypes.byref(p), ms))
    return p.as_tuple(), (ms[0], ms[1], ms[2])


def gp_get_nn_params(ctx) -> Tuple[int, int, int, int, int, int]:
    """(group_span, first_shell, tile_parts, skip_empty, morton_sort, cell_points)."""
    p = gp_nn_params()
    _check(ctx, load_library().gp_get_nn_params(ctx, ctypes.byref(p)))
    return p.as_tuple()


def gp_autotune_nn(ctx, qx, qy, qz, nn_out, reps: int = 2) -> Tuple[Tuple[int, int, int, int, int, int], float]:
    """Time the search grids and NN search shapes on these queries and keep the fastest:
    ((group_span, first_shell, tile_parts, skip_empty, morton_sort, cell_points), ms)."""
    _stream(ctx)
    p, ms = gp_nn_params(), ctypes.c_float(0.0)
    _check(ctx, load_library().gp_autotune_nn(ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32),
                                              _ptr(qz, torch.float32), qx.numel(), _ptr(nn_out, torch.int32),
                                              int(reps), ctypes.byref(p), ctypes.byref(ms)))
    return p.as_tuple(), ms.value


def gp_sample_queries(ctx, seed: int, iteration: int, sigma, sigma_const: float, qx, qy, qz, src_out=None) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_sample_queries(ctx, int(seed), int(iteration), _ptr(sigma, torch.float32),
                                                 float(sigma_const), _ptr(qx, torch.float32),
                                                 _ptr(qy, torch.float32), _ptr(qz, torch.float32),
                                                 _ptr(src_out, torch.int32)))


def _weights(alpha, beta, gamma):
    w = gp_weights()
    w.alpha, w.beta, w.gamma = float(alpha), float(beta), float(gamma)
    return w


def gp_pull_forward(ctx, qx, qy, qz, nn, field, weights, loss_out, n_valid_out) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_pull_forward(
        ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32), _ptr(qz, torch.float32), _ptr(nn, torch.int32),
        qx.numel(), _ptr(field, torch.float32), _weights(*weights), _ptr(loss_out, torch.float64),
        _ptr(n_valid_out, torch.int64)))


def gp_pull_forward_static(ctx, qx, qy, qz, nn, field, weights, loss_out, n_valid_out) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_pull_forward_static(
        ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32), _ptr(qz, torch.float32), _ptr(nn, torch.int32),
        qx.numel(), _ptr(field, torch.float32), _weights(*weights), _ptr(loss_out, torch.float64),
        _ptr(n_valid_out, torch.int64)))


def gp_forward_token(ctx) -> int:
    return int(load_library().gp_forward_token(ctx))


def gp_pull_backward(ctx, qx, qy, qz, nn, field, weights, dloss, grad, forward_token: int) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_pull_backward(
        ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32), _ptr(qz, torch.float32), _ptr(nn, torch.int32),
        qx.numel(), _ptr(field, torch.float32), _weights(*weights), _ptr(dloss, torch.float64),
        _ptr(grad, torch.float32), ctypes.c_uint64(int(forward_token))))


def gp_pull_forward_backward(ctx, qx, qy, qz, nn, field, weights, dloss, loss_out, n_valid_out, grad) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_pull_forward_backward(
        ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32), _ptr(qz, torch.float32), _ptr(nn, torch.int32),
        qx.numel(), _ptr(field, torch.float32), _weights(*weights), _ptr(dloss, torch.float64),
        _ptr(loss_out, torch.float64), _ptr(n_valid_out, torch.int64), _ptr(grad, torch.float32)))


def gp_step(ctx, field, grad, m, v, t: int, lr0: float, decay: float = 0.3, decay_every: int = 400,
            beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_step(ctx, _ptr(field, torch.float32), _ptr(grad, torch.float32),
                                       _ptr(m, torch.float32), _ptr(v, torch.float32), int(t), float(lr0),
                                       float(decay), int(decay_every), float(beta1), float(beta2), float(eps)))


def gp_shape_slots(ctx, n_shapes: int):
    out = (ctypes.c_int64 * (n_shapes + 1))()
    _check(ctx, load_library().gp_shape_slots(ctx, out))
    return list(out)


def gp_export_layout(ctx, vertex_id_of_slot, slot_flags=None) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_export_layout(ctx, _ptr(vertex_id_of_slot, torch.int64),
                                                _ptr(slot_flags, torch.uint8)))


def gp_export_active_cells(ctx, shape: int, device=None) -> torch.Tensor:
    """Sorted linear ids of the M1-band cells of one shape (device int64 tensor)."""
    _stream(ctx)
    lib = load_library()
    n = ctypes.c_int64(0)
    st = lib.gp_export_active_cells(ctx, int(shape), None, 0, ctypes.byref(n))
    if st not in (GP_OK, GP_ERR_CAPACITY):
        _check(ctx, st)
    out = torch.empty(max(n.value, 1), dtype=torch.int64, device=device or "cuda")
    if n.value > 0:
        _check(ctx, lib.gp_export_active_cells(ctx, int(shape), _ptr(out, torch.int64), n.value, ctypes.byref(n)))
    return out[: n.value]


def gp_pull_normals(ctx, qx, qy, qz, nn, field, nx, ny, nz, weight: float, dloss, term_out, grad=None) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_pull_normals(ctx, _ptr(qx, torch.float32), _ptr(qy, torch.float32),
                                               _ptr(qz, torch.float32), _ptr(nn, torch.int32), qx.numel(),
                                               _ptr(field, torch.float32), _ptr(nx, torch.float32),
                                               _ptr(ny, torch.float32), _ptr(nz, torch.float32), float(weight),
                                               _ptr(dloss, torch.float64), _ptr(term_out, torch.float64),
                                               _ptr(grad, torch.float32)))


def gp_extract_surface(ctx, shape: int, field, device=None, method: int = 0):
    """Zero-level-set triangles of one shape: (tri float32 [n, 3, 3], key int64 [n]), key ascending.
    method 0: marching cubes, 1: marching tetrahedra."""
    _stream(ctx)
    lib = load_library()
    n = ctypes.c_int64(0)
    st = lib.gp_extract_surface(ctx, int(shape), _ptr(field, torch.float32), None, None, 0, ctypes.byref(n),
                                int(method))
    if st not in (GP_OK, GP_ERR_CAPACITY):
        _check(ctx, st)
    dev = device or field.device
    tri = torch.empty((max(n.value, 1), 3, 3), dtype=torch.float32, device=dev)
    key = torch.empty(max(n.value, 1), dtype=torch.int64, device=dev)
    if n.value > 0:
        _check(ctx, lib.gp_extract_surface(ctx, int(shape), _ptr(field, torch.float32), _ptr(tri, torch.float32),
                                           _ptr(key, torch.int64), n.value, ctypes.byref(n), int(method)))
    return tri[: n.value], key[: n.value]


def gp_gather_vertices(ctx, dense, field) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_gather_vertices(ctx, _ptr(dense, torch.float32), _ptr(field, torch.float32)))


def gp_scatter_vertices(ctx, field, dense) -> None:
    _stream(ctx)
    _check(ctx, load_library().gp_scatter_vertices(ctx, _ptr(field, torch.float32), _ptr(dense, torch.float32)))


def gp_init_sphere(ctx, centre: Sequence[Sequence[float]], radius: Sequence[float], field) -> None:
    _stream(ctx)
    n = len(radius)
    c = (ctypes.c_double * (3 * n))(*[float(x) for row in centre for x in row])
    r = (ctypes.c_double * n)(*[float(x) for x in radius])
    _check(ctx, load_library().gp_init_sphere(ctx, c, r, _ptr(field, torch.float32)))


def gp_timing_enable(ctx, enable: bool = True) -> None:
    _check(ctx, load_library().gp_timing_enable(ctx, 1 if enable else 0))


def gp_timing_report(ctx) -> dict:
    """{kernel name: (launches, total ms)} since the last report."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(ctx, load_library().gp_timing_report(ctx, buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out
