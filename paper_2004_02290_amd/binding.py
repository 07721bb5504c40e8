"""Python binding of libghn, the gfx950 Grid Hashing Neighborhood KNN library.

Argument marshalling only: every step of build and predict runs in the HIP
kernels of libghn.so.  The module-level functions carry the names of the C
entry points (see include/ghn.h); `Index` is a small owner object around a
handle.  Tensors must be on the GPU; the current torch stream is used unless
a stream is passed.  Importing this module fails loudly if libghn.so has not
been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
from typing import Optional, Sequence, Union

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libghn.so")

GHN_OK = 0
STATUS = {0: "GHN_OK", -1: "GHN_E_INVALID_ARG", -2: "GHN_E_UNSUPPORTED", -3: "GHN_E_K_GT_N",
          -4: "GHN_E_NONFINITE", -5: "GHN_E_KEY_OVERFLOW", -6: "GHN_E_WORKSPACE", -7: "GHN_E_HIP",
          -8: "GHN_E_NOMEM"}
GHN_F32, GHN_BF16 = 0, 1
GHN_CLASSIFY, GHN_REGRESS = 0, 1
GHN_STOP_EXACT, GHN_STOP_PAPER = 0, 1
GHN_PREC_FP32, GHN_PREC_BF16_MFMA = 0, 1
GHN_FLAG_NO_PRUNE, GHN_FLAG_NO_SORT, GHN_FLAG_MEDIAN, GHN_FLAG_RING_GROW = 1, 2, 4, 8
GHN_WALK_SHORT = 1
GHN_K_MAX, GHN_F_MAX = 64, 32

GHN_LOOKUP_AUTO, GHN_LOOKUP_DENSE, GHN_LOOKUP_TREE, GHN_LOOKUP_HASH = -1, 0, 1, 2

P_ = ctypes.c_void_p

EXPORTED = ["ghn_build", "ghn_build_ex", "ghn_index_get_info", "ghn_destroy", "ghn_predict_workspace_bytes", "ghn_predict",
            "ghn_query_order_workspace_bytes", "ghn_query_order", "ghn_batch_workspace_bytes", "ghn_batch_prepare",
            "ghn_predict_batched", "ghn_batch_destroy", "ghn_autotune", "ghn_cell_measure", "ghn_bruteforce",
            "ghn_index_save_bytes", "ghn_index_save", "ghn_index_load", "ghn_insert", "ghn_screen_error",
            "ghn_predict_noalloc", "ghn_build_workspace_bytes", "ghn_index_bytes", "ghn_index_bytes_for",
            "ghn_build_into", "ghn_batch_workspace_bytes_for", "ghn_index_cells", "ghn_walk_faults",
            "ghn_last_error"]
GHN_NOALLOC_WS_BYTES = 64 << 20


class GHNError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, message))
        self.code = code
        self.message = message


class ghn_index_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("f", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("task", ctypes.c_int32), ("lookup", ctypes.c_int32), ("num_cells", ctypes.c_int64),
                ("box_cells", ctypes.c_int64), ("max_occupancy", ctypes.c_int64),
                ("cell_min", ctypes.c_int32 * GHN_F_MAX), ("cell_max", ctypes.c_int32 * GHN_F_MAX),
                ("cell_width", ctypes.c_float * GHN_F_MAX), ("origin", ctypes.c_float * GHN_F_MAX),
                ("device_bytes", ctypes.c_size_t)]


class ghn_predict_opts(ctypes.Structure):
    _fields_ = [("stop", ctypes.c_int32), ("prec", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("out_stop_layer", ctypes.c_void_p), ("out_cands", ctypes.c_void_p),
                ("out_probes", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("group_levels", ctypes.c_int32), ("walk_event_begin", ctypes.c_void_p),
                ("walk_event_end", ctypes.c_void_p), ("out_rerank", ctypes.c_void_p),
                ("ring_step", ctypes.c_int32), ("group_size", ctypes.c_int32), ("tile_width", ctypes.c_int32)]


class ghn_batch_item(ctypes.Structure):
    _fields_ = [("index", ctypes.c_void_p), ("queries", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("k", ctypes.c_int32), ("out_idx", ctypes.c_void_p), ("out_d2", ctypes.c_void_p),
                ("out_pred", ctypes.c_void_p)]


class ghn_tune_trial(ctypes.Structure):
    _fields_ = [("cell_width", ctypes.c_float), ("lookup", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("group_levels", ctypes.c_int32), ("flags", ctypes.c_uint32), ("ring_step", ctypes.c_int32),
                ("group_size", ctypes.c_int32), ("tile_width", ctypes.c_int32), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libghn.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_2004_02290_amd._build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.ghn_build.argtypes = [P, I64, I32, I32, P, I32, P, I32, P, P, ctypes.POINTER(P)]
    L.ghn_build.restype = ctypes.c_int
    L.ghn_build_ex.argtypes = [P, I64, I32, I32, P, I32, P, I32, P, P, P, ctypes.POINTER(P)]
    L.ghn_build_ex.restype = ctypes.c_int
    L.ghn_build_workspace_bytes.argtypes = [I64, I32]
    L.ghn_build_workspace_bytes.restype = SZ
    L.ghn_index_bytes.argtypes = [I64, I32, I32, I32]
    L.ghn_index_bytes.restype = SZ
    L.ghn_index_bytes_for.argtypes = [P, I64, I32, I32, I32, P, I32, P, P, P, SZ, P, ctypes.POINTER(SZ)]
    L.ghn_index_bytes_for.restype = ctypes.c_int
    L.ghn_build_into.argtypes = [P, I64, I32, I32, P, I32, P, I32, P, P, P, SZ, P, SZ, P, ctypes.POINTER(P)]
    L.ghn_build_into.restype = ctypes.c_int
    L.ghn_index_cells.argtypes = [P, P, P, P, P]
    L.ghn_index_cells.restype = ctypes.c_int
    L.ghn_walk_faults.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.c_int, P]
    L.ghn_walk_faults.restype = ctypes.c_int
    L.ghn_index_get_info.argtypes = [P, ctypes.POINTER(ghn_index_info)]
    L.ghn_index_get_info.restype = ctypes.c_int
    L.ghn_destroy.argtypes = [P]
    L.ghn_destroy.restype = None
    L.ghn_predict_workspace_bytes.argtypes = [P, I64, I32, ctypes.POINTER(ghn_predict_opts)]
    L.ghn_predict_workspace_bytes.restype = SZ
    L.ghn_predict.argtypes = [P, P, I64, I32, ctypes.POINTER(ghn_predict_opts), P, P, P, P, SZ, P]
    L.ghn_predict.restype = ctypes.c_int
    L.ghn_query_order_workspace_bytes.argtypes = [I64]
    L.ghn_query_order_workspace_bytes.restype = SZ
    L.ghn_query_order.argtypes = [P, P, I64, P, P, SZ, P]
    L.ghn_query_order.restype = ctypes.c_int
    L.ghn_batch_workspace_bytes.argtypes = [I32]
    L.ghn_batch_workspace_bytes.restype = SZ
    L.ghn_batch_workspace_bytes_for.argtypes = [ctypes.POINTER(ghn_batch_item), I32, ctypes.POINTER(ghn_predict_opts)]
    L.ghn_batch_workspace_bytes_for.restype = SZ
    L.ghn_batch_prepare.argtypes = [ctypes.POINTER(ghn_batch_item), I32, ctypes.POINTER(ghn_predict_opts), P, SZ, P,
                                    ctypes.POINTER(P)]
    L.ghn_batch_prepare.restype = ctypes.c_int
    L.ghn_predict_batched.argtypes = [P, P]
    L.ghn_predict_batched.restype = ctypes.c_int
    L.ghn_batch_destroy.argtypes = [P]
    L.ghn_batch_destroy.restype = None
    L.ghn_autotune.argtypes = [P, I64, I32, I32, P, I32, P, I64, I32, I32, P, I32, ctypes.POINTER(ghn_tune_trial),
                               ctypes.POINTER(ghn_tune_trial), I32, ctypes.POINTER(I32), P]
    L.ghn_autotune.restype = ctypes.c_int
    L.ghn_predict_noalloc.argtypes = [P, P, I64, I32, ctypes.POINTER(ghn_predict_opts), P, P, P, P]
    L.ghn_predict_noalloc.restype = ctypes.c_int
    L.ghn_bruteforce.argtypes = [P, P, I64, I32, ctypes.POINTER(ghn_predict_opts), P, P, P, P, SZ, P]
    L.ghn_bruteforce.restype = ctypes.c_int
    L.ghn_index_save_bytes.argtypes = [P]
    L.ghn_index_save_bytes.restype = SZ
    L.ghn_index_save.argtypes = [P, P, SZ, P]
    L.ghn_index_save.restype = ctypes.c_int
    L.ghn_index_load.argtypes = [P, SZ, P, ctypes.POINTER(P)]
    L.ghn_index_load.restype = ctypes.c_int
    L.ghn_insert.argtypes = [P, P, I64, I32, P, P]
    L.ghn_insert.restype = ctypes.c_int
    L.ghn_screen_error.argtypes = [P, P, I64, I64, P, P, P]
    L.ghn_screen_error.restype = ctypes.c_int
    L.ghn_cell_measure.argtypes = [P, I64, I32, I32, P, P, P, P]
    L.ghn_cell_measure.restype = ctypes.c_int
    L.ghn_last_error.argtypes = []
    L.ghn_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def ghn_last_error() -> str:
    return _lib.ghn_last_error().decode()


def _check(code: int):
    if code != GHN_OK:
        raise GHNError(code, ghn_last_error())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class ghn_build_opts(ctypes.Structure):
    _fields_ = [("lookup", ctypes.c_int32)]


def ghn_build(points: torch.Tensor, targets: torch.Tensor, task: int,
              cell_width: Union[float, Sequence[float]], origin: Optional[Sequence[float]] = None,
              stream=None) -> ctypes.c_void_p:
    """ghn_build: points n x f (float32, or bfloat16 -> stored as bf16), targets n (int32 | float32)."""
    return ghn_build_ex(points, targets, task, cell_width, origin, None, stream)


def ghn_build_ex(points: torch.Tensor, targets: torch.Tensor, task: int,
                 cell_width: Union[float, Sequence[float]], origin: Optional[Sequence[float]] = None,
                 lookup: Optional[int] = None, stream=None) -> ctypes.c_void_p:
    """ghn_build_ex: as ghn_build, with the cell lookup structure chosen (GHN_LOOKUP_*)."""
    dtype = _points_dtype(points)
    n, f = points.shape
    want = torch.int32 if task == GHN_CLASSIFY else torch.float32
    if targets.dtype != want or targets.numel() != n:
        raise ValueError("targets must be %s with n entries" % want)
    w, nw, o = _widths(cell_width, origin)
    h = ctypes.c_void_p()
    opts = None if lookup is None else ctypes.byref(ghn_build_opts(int(lookup)))
    _check(_lib.ghn_build_ex(_ptr(points), n, f, dtype, _ptr(targets), task, w, nw, o, opts, _stream(stream),
                             ctypes.byref(h)))
    return h


def _widths(cell_width, origin):
    w = (ctypes.c_float * GHN_F_MAX)()
    ws = [float(cell_width)] if isinstance(cell_width, (int, float)) else [float(x) for x in cell_width]
    for i, x in enumerate(ws):
        w[i] = x
    o = None
    if origin is not None:
        o = (ctypes.c_float * GHN_F_MAX)()
        for i, x in enumerate(origin):
            o[i] = float(x)
    return w, len(ws), o


def _points_dtype(points: torch.Tensor) -> int:
    if points.dim() != 2:
        raise ValueError("points must be n x f")
    if points.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("points must be float32 or bfloat16")
    return GHN_BF16 if points.dtype == torch.bfloat16 else GHN_F32


def ghn_build_workspace_bytes(n: int, f: int) -> int:
    return int(_lib.ghn_build_workspace_bytes(n, f))


def ghn_index_bytes(n: int, f: int, dtype: int = GHN_F32, task: int = GHN_CLASSIFY) -> int:
    return int(_lib.ghn_index_bytes(n, f, dtype, task))


def ghn_index_bytes_for(points: torch.Tensor, task: int, cell_width, ws: torch.Tensor, origin=None,
                        lookup: Optional[int] = None, stream=None) -> int:
    """ghn_index_bytes_for: index storage bytes for these points and widths (runs the cell-range pass in ws)."""
    dtype = _points_dtype(points)
    n, f = points.shape
    w, nw, o = _widths(cell_width, origin)
    opts = None if lookup is None else ctypes.byref(ghn_build_opts(int(lookup)))
    out = ctypes.c_size_t(0)
    _check(_lib.ghn_index_bytes_for(_ptr(points), n, f, dtype, task, w, nw, o, opts, _ptr(ws),
                                    ws.numel() * ws.element_size(), _stream(stream), ctypes.byref(out)))
    return int(out.value)


def ghn_build_into(points: torch.Tensor, targets: torch.Tensor, task: int, cell_width, storage: torch.Tensor,
                   ws: torch.Tensor, origin=None, lookup: Optional[int] = None, stream=None) -> ctypes.c_void_p:
    """ghn_build_into: the build with the index in `storage` and temporaries in `ws` (uint8 GPU tensors)."""
    dtype = _points_dtype(points)
    n, f = points.shape
    want = torch.int32 if task == GHN_CLASSIFY else torch.float32
    if targets.dtype != want or targets.numel() != n:
        raise ValueError("targets must be %s with n entries" % want)
    w, nw, o = _widths(cell_width, origin)
    opts = None if lookup is None else ctypes.byref(ghn_build_opts(int(lookup)))
    h = ctypes.c_void_p()
    _check(_lib.ghn_build_into(_ptr(points), n, f, dtype, _ptr(targets), task, w, nw, o, opts, _ptr(storage),
                               storage.numel() * storage.element_size(), _ptr(ws), ws.numel() * ws.element_size(),
                               _stream(stream), ctypes.byref(h)))
    return h


def ghn_index_get_info(handle) -> ghn_index_info:
    info = ghn_index_info()
    _check(_lib.ghn_index_get_info(handle, ctypes.byref(info)))
    return info


def ghn_index_cells(handle, stream=None):
    """ghn_index_cells: (ids num_cells x f int32, counts num_cells int64, point_cell n int32) GPU tensors."""
    info = ghn_index_get_info(handle)
    ids = torch.empty((info.num_cells, info.f), dtype=torch.int32, device="cuda")
    counts = torch.empty(info.num_cells, dtype=torch.int64, device="cuda")
    point_cell = torch.empty(info.n, dtype=torch.int32, device="cuda")
    _check(_lib.ghn_index_cells(handle, _ptr(ids), _ptr(counts), _ptr(point_cell), _stream(stream)))
    return ids, counts, point_cell


def ghn_walk_faults(clear=False, stream=None) -> int:
    """ghn_walk_faults: the current device's walk fault bits (GHN_WALK_SHORT), after
    waiting for `stream`; clear resets them."""
    v = ctypes.c_uint32(0)
    _check(_lib.ghn_walk_faults(ctypes.byref(v), int(bool(clear)), _stream(stream)))
    return v.value


def ghn_destroy(handle) -> None:
    _lib.ghn_destroy(handle)


def _event(ev):
    """Raw hipEvent_t of a torch.cuda.Event (recorded once so that it exists), or None."""
    if ev is None:
        return None
    if not ev.cuda_event:
        ev.record()
    return ctypes.c_void_p(ev.cuda_event)


def _opts(stop, prec, flags, out_stop_layer=None, out_cands=None, out_probes=None, order=None,
          group_levels=-1, walk_events=None, out_rerank=None, ring_step=0, group_size=0,
          tile_width=0) -> ghn_predict_opts:
    ev0, ev1 = walk_events if walk_events is not None else (None, None)
    return ghn_predict_opts(int(stop), int(prec), int(flags), _ptr(out_stop_layer), _ptr(out_cands),
                            _ptr(out_probes), _ptr(order), int(group_levels), _event(ev0), _event(ev1),
                            _ptr(out_rerank), int(ring_step), int(group_size), int(tile_width))


def ghn_predict_workspace_bytes(handle, m: int, k: int, stop=GHN_STOP_EXACT, prec=GHN_PREC_FP32, flags=0,
                                group_levels=-1) -> int:
    o = _opts(stop, prec, flags, group_levels=group_levels)
    return int(_lib.ghn_predict_workspace_bytes(handle, m, k, ctypes.byref(o)))


def ghn_predict(handle, queries: torch.Tensor, k: int, out_idx: torch.Tensor, out_pred: torch.Tensor,
                out_d2: Optional[torch.Tensor] = None, stop=GHN_STOP_EXACT, prec=GHN_PREC_FP32, flags=0,
                out_stop_layer: Optional[torch.Tensor] = None, out_cands: Optional[torch.Tensor] = None,
                out_probes: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                order: Optional[torch.Tensor] = None, group_levels: int = -1, stream=None,
                walk_events=None, out_rerank: Optional[torch.Tensor] = None, ring_step: int = 0,
                group_size: int = 0, tile_width: int = 0) -> None:
    """ghn_predict into caller-provided outputs (int64 idx m x k, pred m, optional float64 d2 m x k).

    walk_events: optional (begin, end) pair of torch.cuda.Event recorded around the walk kernel."""
    m = queries.shape[0]
    o = _opts(stop, prec, flags, out_stop_layer, out_cands, out_probes, order, group_levels, walk_events,
              out_rerank, ring_step, group_size, tile_width)
    ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.ghn_predict(handle, _ptr(queries), m, k, ctypes.byref(o), _ptr(out_idx), _ptr(out_d2),
                            _ptr(out_pred), _ptr(ws), ws_bytes, _stream(stream)))


def ghn_predict_noalloc(handle, queries: torch.Tensor, k: int, out_idx: torch.Tensor, out_pred: torch.Tensor,
                        out_d2: Optional[torch.Tensor] = None, stop=GHN_STOP_EXACT, prec=GHN_PREC_FP32, flags=0,
                        out_stop_layer: Optional[torch.Tensor] = None, group_levels: int = -1, stream=None) -> None:
    """ghn_predict_noalloc: ghn_predict with the library's own per-GPU workspace array (no allocation)."""
    m = queries.shape[0]
    o = _opts(stop, prec, flags, out_stop_layer, group_levels=group_levels)
    _check(_lib.ghn_predict_noalloc(handle, _ptr(queries), m, k, ctypes.byref(o), _ptr(out_idx), _ptr(out_d2),
                                    _ptr(out_pred), _stream(stream)))


def ghn_bruteforce(handle, queries: torch.Tensor, k: int, out_idx: torch.Tensor, out_pred: torch.Tensor,
                   out_d2: Optional[torch.Tensor] = None, flags=0, out_cands: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, stream=None, walk_events=None) -> None:
    """ghn_bruteforce: exhaustive KNN over the index's points (bf16 screen + FP64 re-rank)."""
    m = queries.shape[0]
    o = _opts(GHN_STOP_EXACT, GHN_PREC_BF16_MFMA, flags, None, out_cands, None, None, -1, walk_events)
    ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.ghn_bruteforce(handle, _ptr(queries), m, k, ctypes.byref(o), _ptr(out_idx), _ptr(out_d2),
                               _ptr(out_pred), _ptr(ws), ws_bytes, _stream(stream)))


def ghn_query_order_workspace_bytes(m: int) -> int:
    return int(_lib.ghn_query_order_workspace_bytes(m))


def ghn_query_order(handle, queries: torch.Tensor, out_order: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    """ghn_query_order: spatial walk order (m uint32, passed as an int32 tensor) of a query batch."""
    m = queries.shape[0]
    ws_bytes = ws.numel() * ws.element_size()
    _check(_lib.ghn_query_order(handle, _ptr(queries), m, _ptr(out_order), _ptr(ws), ws_bytes, _stream(stream)))


def ghn_batch_workspace_bytes(n_items: int) -> int:
    return int(_lib.ghn_batch_workspace_bytes(n_items))


def _batch_items(items):
    arr = (ghn_batch_item * len(items))()
    for i, (h, q, k, oi, op, od) in enumerate(items):
        arr[i] = ghn_batch_item(h.value if isinstance(h, ctypes.c_void_p) else h, _ptr(q), q.shape[0], int(k),
                                _ptr(oi), _ptr(od), _ptr(op))
    return arr


def ghn_batch_workspace_bytes_for(items, stop=GHN_STOP_EXACT, prec=GHN_PREC_FP32, flags=0, group_levels=-1) -> int:
    """ghn_batch_workspace_bytes_for: workspace of a batch of these items (as ghn_batch_prepare's)."""
    o = _opts(stop, prec, flags, group_levels=group_levels)
    return int(_lib.ghn_batch_workspace_bytes_for(_batch_items(items), len(items), ctypes.byref(o)))


def ghn_batch_prepare(items, ws: torch.Tensor, stop=GHN_STOP_EXACT, flags=0, stream=None, prec=GHN_PREC_FP32,
                      group_levels=-1, ring_step=0, group_size=0, tile_width=0) -> ctypes.c_void_p:
    """ghn_batch_prepare: items = [(handle, queries, k, out_idx, out_pred, out_d2 or None), ...]."""
    arr = _batch_items(items)
    o = _opts(stop, prec, flags, group_levels=group_levels, ring_step=ring_step, group_size=group_size,
              tile_width=tile_width)
    out = ctypes.c_void_p()
    _check(_lib.ghn_batch_prepare(arr, len(items), ctypes.byref(o), _ptr(ws), ws.numel() * ws.element_size(),
                                  _stream(stream), ctypes.byref(out)))
    return out


def ghn_predict_batched(batch, stream=None) -> None:
    _check(_lib.ghn_predict_batched(batch, _stream(stream)))


def ghn_batch_destroy(batch) -> None:
    _lib.ghn_batch_destroy(batch)


def ghn_autotune(points: torch.Tensor, targets: torch.Tensor, task: int, queries: torch.Tensor, k: int,
                 stop=GHN_STOP_EXACT, widths=None, max_trials: int = 256, stream=None):
    """ghn_autotune: returns (best trial dict, list of trial dicts)."""
    n, f = points.shape
    dtype = GHN_BF16 if points.dtype == torch.bfloat16 else GHN_F32
    w = None
    nw = 0
    if widths is not None:
        ws_ = [float(x) for x in np.atleast_1d(widths)]
        w = (ctypes.c_float * len(ws_))(*ws_)
        nw = len(ws_)
    best = ghn_tune_trial()
    trials = (ghn_tune_trial * max_trials)()
    nt = ctypes.c_int32(0)
    _check(_lib.ghn_autotune(_ptr(points), n, f, dtype, _ptr(targets), task, _ptr(queries), queries.shape[0], int(k),
                             int(stop), w, nw, ctypes.byref(best), trials, max_trials, ctypes.byref(nt),
                             _stream(stream)))
    return best.as_dict(), [trials[i].as_dict() for i in range(min(nt.value, max_trials))]


def ghn_index_save(handle, stream=None) -> bytes:
    """ghn_index_save: the index as bytes (header, points in original order, targets)."""
    nbytes = int(_lib.ghn_index_save_bytes(handle))
    buf = ctypes.create_string_buffer(nbytes)
    _check(_lib.ghn_index_save(handle, ctypes.cast(buf, P_), nbytes, _stream(stream)))
    return buf.raw


def ghn_index_load(data: bytes, stream=None):
    """ghn_index_load: a handle rebuilt from ghn_index_save's bytes."""
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(data, len(data))
    _check(_lib.ghn_index_load(ctypes.cast(buf, P_), len(data), _stream(stream), ctypes.byref(h)))
    return h


def ghn_insert(handle, points: torch.Tensor, targets: torch.Tensor, stream=None) -> None:
    """ghn_insert: append points (n_new x f, float32 or bfloat16) and their targets to an index."""
    dtype = GHN_BF16 if points.dtype == torch.bfloat16 else GHN_F32
    _check(_lib.ghn_insert(handle, _ptr(points), points.shape[0], dtype, _ptr(targets), _stream(stream)))


def ghn_screen_error(handle, queries: torch.Tensor, sample: int = 4096, stream=None):
    """ghn_screen_error: per query (max |s - d|, max |s - d| / (|q'|^2 + |x'|^2)) as float32 GPU tensors."""
    m = queries.shape[0]
    ea = torch.empty(m, dtype=torch.float32, device=queries.device)
    er = torch.empty(m, dtype=torch.float32, device=queries.device)
    _check(_lib.ghn_screen_error(handle, _ptr(queries), m, int(sample), _ptr(ea), _ptr(er), _stream(stream)))
    return ea, er


def ghn_cell_measure(points: torch.Tensor, stream=None):
    """ghn_cell_measure: the paper's cell measurements -> (width float32[f], origin float32[f], splits int64[f])."""
    n, f = points.shape
    dtype = GHN_BF16 if points.dtype == torch.bfloat16 else GHN_F32
    w = np.empty(f, dtype=np.float32)
    o = np.empty(f, dtype=np.float32)
    sp = np.empty(f, dtype=np.int64)
    _check(_lib.ghn_cell_measure(_ptr(points), n, f, dtype, w.ctypes.data_as(P_), o.ctypes.data_as(P_),
                                 sp.ctypes.data_as(P_), _stream(stream)))
    return w, o, sp


class Index:
    """Owner of a built index (build on construction, free on close / garbage collection)."""

    def __init__(self, points: torch.Tensor, targets: torch.Tensor, task: int,
                 cell_width: Union[float, Sequence[float]], origin=None, lookup: Optional[int] = None, stream=None,
                 torch_storage: bool = False):
        """torch_storage: the index lives in a torch tensor (ghn_build_into) instead of library memory."""
        self.task = task
        self.storage = None
        if torch_storage:
            n, f = points.shape
            ws = torch.empty(ghn_build_workspace_bytes(n, f), dtype=torch.uint8, device=points.device)
            nbytes = ghn_index_bytes_for(points, task, cell_width, ws, origin, lookup, stream)
            self.storage = torch.empty(nbytes, dtype=torch.uint8, device=points.device)
            self.handle = ghn_build_into(points, targets, task, cell_width, self.storage, ws, origin, lookup, stream)
        else:
            self.handle = ghn_build_ex(points, targets, task, cell_width, origin, lookup, stream)
        self.info = ghn_index_get_info(self.handle)

    def predict(self, queries: torch.Tensor, k: int, stop=GHN_STOP_EXACT, prec=GHN_PREC_FP32, flags=0,
                with_d2: bool = True, with_stats: bool = False, group_levels: int = -1, stream=None,
                ring_step: int = 0, group_size: int = 0, tile_width: int = 0):
        """Returns dict(idx, pred[, d2][, stop_layer, cands]) as GPU tensors."""
        dev = queries.device
        m = queries.shape[0]
        out = dict(idx=torch.empty((m, k), dtype=torch.int64, device=dev),
                   pred=torch.empty(m, dtype=torch.int32 if self.task == GHN_CLASSIFY else torch.float32,
                                    device=dev))
        if with_d2:
            out["d2"] = torch.empty((m, k), dtype=torch.float64, device=dev)
        if with_stats:
            out["stop_layer"] = torch.empty(m, dtype=torch.int32, device=dev)
            out["cands"] = torch.empty(m, dtype=torch.int64, device=dev)
            out["probes"] = torch.empty(m, dtype=torch.int64, device=dev)
            out["rerank"] = torch.empty(m, dtype=torch.int64, device=dev)
        nbytes = ghn_predict_workspace_bytes(self.handle, m, k, stop, prec, flags, group_levels)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev) if nbytes else None
        ghn_predict(self.handle, queries, k, out["idx"], out["pred"], out.get("d2"), stop, prec, flags,
                    out.get("stop_layer"), out.get("cands"), out.get("probes"), ws, None, group_levels, stream,
                    out_rerank=out.get("rerank"), ring_step=ring_step, group_size=group_size,
                    tile_width=tile_width)
        return out

    @classmethod
    def load(cls, data: bytes, stream=None) -> "Index":
        """An index rebuilt from save()'s bytes."""
        self = cls.__new__(cls)
        self.handle = ghn_index_load(data, stream)
        self.info = ghn_index_get_info(self.handle)
        self.task = self.info.task
        return self

    def save(self, stream=None) -> bytes:
        return ghn_index_save(self.handle, stream)

    def insert(self, points: torch.Tensor, targets: torch.Tensor, stream=None) -> None:
        if points.dim() != 2 or points.shape[1] != self.info.f or targets.shape[0] != points.shape[0]:
            raise ValueError("insert: points must be n_new x %d with n_new targets" % self.info.f)
        ghn_insert(self.handle, points, targets, stream)
        self.info = ghn_index_get_info(self.handle)

    def bruteforce(self, queries: torch.Tensor, k: int, flags=0, with_d2: bool = True, with_stats: bool = False,
                   stream=None):
        """Exhaustive KNN over the index's points; returns dict(idx, pred[, d2][, cands]) as GPU tensors."""
        dev = queries.device
        m = queries.shape[0]
        out = dict(idx=torch.empty((m, k), dtype=torch.int64, device=dev),
                   pred=torch.empty(m, dtype=torch.int32 if self.task == GHN_CLASSIFY else torch.float32,
                                    device=dev))
        if with_d2:
            out["d2"] = torch.empty((m, k), dtype=torch.float64, device=dev)
        if with_stats:
            out["cands"] = torch.empty(m, dtype=torch.int64, device=dev)
        nbytes = ghn_predict_workspace_bytes(self.handle, m, k, GHN_STOP_EXACT, GHN_PREC_BF16_MFMA, flags)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev) if nbytes else None
        ghn_bruteforce(self.handle, queries, k, out["idx"], out["pred"], out.get("d2"), flags, out.get("cands"), ws,
                       stream)
        return out

    def close(self):
        if getattr(self, "handle", None):
            ghn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
