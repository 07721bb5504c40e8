"""Python access to the GHN CPU oracle (test infrastructure only).

The oracle is a plain FP64 C++ implementation of the paper's method (cell
sampling by Eq. 1 and Algorithm 1, layer-by-layer exploration of Section III-B)
plus brute-force KNN.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may use it; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ghn_oracle.cpp")
LIB = os.path.join(HERE, "libghn_oracle.so")

CLASSIFY, REGRESS = 0, 1
REGRESS_MEDIAN = 2  # regression with the median of the k targets
STOP_EXACT, STOP_PAPER = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP over queries)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        I64, I32 = ctypes.c_int64, ctypes.c_int32
        L.ghn_oracle_cells.argtypes = [P, I64, I32, P, I32, P, P]
        L.ghn_oracle_cells.restype = ctypes.c_int
        L.ghn_oracle_count_cells.argtypes = [P, I64, I32, P, I32, P]
        L.ghn_oracle_count_cells.restype = I64
        L.ghn_oracle_bruteforce.argtypes = [P, I64, I32, P, I32, P, I64, I32, P, P, P, I32]
        L.ghn_oracle_bruteforce.restype = ctypes.c_int
        L.ghn_oracle_grid_build.argtypes = [P, I64, I32, P, I32, P, I32, P]
        L.ghn_oracle_grid_build.restype = P
        L.ghn_oracle_grid_num_cells.argtypes = [P]
        L.ghn_oracle_grid_num_cells.restype = I64
        L.ghn_oracle_grid_cells.argtypes = [P, P, P]
        L.ghn_oracle_grid_cells.restype = ctypes.c_int
        L.ghn_oracle_grid_predict.argtypes = [P, P, I64, I32, I32, P, P, P, P, P, P, I32]
        L.ghn_oracle_grid_predict.restype = ctypes.c_int
        L.ghn_oracle_grid_trace.argtypes = [P, P, I32, I32, P, P, I32]
        L.ghn_oracle_grid_trace.restype = I32
        L.ghn_oracle_grid_free.argtypes = [P]
        L.ghn_oracle_grid_free.restype = None
        L.ghn_oracle_cell_measure.argtypes = [P, I64, I32, P, P, P]
        L.ghn_oracle_cell_measure.restype = I32
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _widths(widths, f):
    w = np.atleast_1d(np.asarray(widths, dtype=np.float32))
    if w.size not in (1, f):
        raise ValueError("widths must be a scalar or have f entries")
    return np.ascontiguousarray(w), int(w.size)


def _targets(targets, task):
    return np.ascontiguousarray(targets, dtype=np.int32 if task == CLASSIFY else np.float32)


def cell_measure(points):
    """The paper's cell measurement rule: (width float32[f], origin float32[f], splits int64[f])."""
    x = _f32(points)
    n, f = x.shape
    w = np.empty(f, dtype=np.float32)
    o = np.empty(f, dtype=np.float32)
    s = np.empty(f, dtype=np.int64)
    if lib().ghn_oracle_cell_measure(_p(x), n, f, _p(w), _p(o), _p(s)) != 0:
        raise ValueError("oracle cell_measure rejected its arguments")
    return w, o, s


def cells(points, widths, origin=None) -> np.ndarray:
    """Cell coordinates (Eq. 1) of every point, n x f int64."""
    x = _f32(points)
    n, f = x.shape
    w, nw = _widths(widths, f)
    o = None if origin is None else _f32(origin)
    out = np.empty((n, f), dtype=np.int64)
    lib().ghn_oracle_cells(_p(x), n, f, _p(w), nw, _p(o), _p(out))
    return out


def count_cells(points, widths, origin=None) -> int:
    x = _f32(points)
    n, f = x.shape
    w, nw = _widths(widths, f)
    o = None if origin is None else _f32(origin)
    return int(lib().ghn_oracle_count_cells(_p(x), n, f, _p(w), nw, _p(o)))


def _pred_array(task, m):
    return np.empty(m, dtype=np.int32 if task == CLASSIFY else np.float32)


def bruteforce(points, targets, task, queries, k, nthreads: int = 0):
    """Plain KNN: returns (idx m x k int64, d2 m x k float64, pred m)."""
    x, q = _f32(points), _f32(queries)
    n, f = x.shape
    m = q.shape[0]
    t = _targets(targets, task)
    idx = np.empty((m, k), dtype=np.int64)
    d2 = np.empty((m, k), dtype=np.float64)
    pred = _pred_array(task, m)
    rc = lib().ghn_oracle_bruteforce(_p(x), n, f, _p(t), task, _p(q), m, k, _p(idx), _p(d2), _p(pred),
                                     nthreads)
    if rc != 0:
        raise ValueError("oracle bruteforce rejected its arguments (k must be in [1, n])")
    return idx, d2, pred


class Grid:
    """Algorithm 1's hash table plus the Section III-B exploration."""

    def __init__(self, points, targets, task, widths, origin=None):
        x = _f32(points)
        n, f = x.shape
        self.n, self.f, self.task = n, f, task
        w, nw = _widths(widths, f)
        o = None if origin is None else _f32(origin)
        t = _targets(targets, task)
        self._h = lib().ghn_oracle_grid_build(_p(x), n, f, _p(t), task, _p(w), nw, _p(o))

    @property
    def num_cells(self) -> int:
        return int(lib().ghn_oracle_grid_num_cells(self._h))

    def cells(self):
        nc = self.num_cells
        ids = np.empty((nc, self.f), dtype=np.int64)
        counts = np.empty(nc, dtype=np.int64)
        lib().ghn_oracle_grid_cells(self._h, _p(ids), _p(counts))
        return ids, counts

    def predict(self, queries, k, stop=STOP_EXACT, nthreads: int = 0):
        """Returns dict(idx, d2, pred, stop_layer, cells, cands)."""
        q = _f32(queries)
        m = q.shape[0]
        idx = np.empty((m, k), dtype=np.int64)
        d2 = np.empty((m, k), dtype=np.float64)
        pred = _pred_array(self.task, m)
        sl = np.empty(m, dtype=np.int32)
        cells = np.empty(m, dtype=np.int64)
        cands = np.empty(m, dtype=np.int64)
        rc = lib().ghn_oracle_grid_predict(self._h, _p(q), m, k, stop, _p(idx), _p(d2), _p(pred), _p(sl),
                                           _p(cells), _p(cands), nthreads)
        if rc != 0:
            raise ValueError("oracle grid predict rejected its arguments (k must be in [1, n])")
        return dict(idx=idx, d2=d2, pred=pred, stop_layer=sl, cells=cells, cands=cands)

    def trace(self, query, k, stop=STOP_EXACT, max_layers: int = 64):
        """Per-layer (cells visited, buffer updated) of one query, plus the stop layer."""
        q = _f32(query).reshape(-1)
        lc = np.zeros(max_layers, dtype=np.int64)
        lu = np.zeros(max_layers, dtype=np.int32)
        stop_layer = lib().ghn_oracle_grid_trace(self._h, _p(q), k, stop, _p(lc), _p(lu), max_layers)
        return int(stop_layer), lc, lu

    def close(self):
        if getattr(self, "_h", None):
            lib().ghn_oracle_grid_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
