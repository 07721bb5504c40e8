"""The C ABI library loads, exports every entry point declared in include/ghn.h, and
rejects bad arguments on the host (before any GPU work) with the documented codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ghn.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ghn_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ghn():
    from paper_2004_02290_amd import binding
    return binding


def test_every_declared_symbol_is_exported(ghn):
    names = _declared()
    assert "ghn_build" in names and "ghn_predict" in names
    lib = ctypes.CDLL(ghn.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(ghn.EXPORTED) == names


def test_struct_sizes_match_header(ghn):
    # ghn_index_info: 8+4+4+4+4+8+8+8 + 4*32*4 + 8 bytes
    # ghn_predict_opts: 3*4 + pad + 4*8 + 4 + pad + 3*8
    assert ctypes.sizeof(ghn.ghn_index_info) == 48 + 4 * 32 * 4 + 8
    assert ctypes.sizeof(ghn.ghn_predict_opts) == 80
    assert ctypes.sizeof(ghn.ghn_batch_item) == 56  # 3 pointers/ints of 8, k + pad, 3 pointers
    assert ctypes.sizeof(ghn.ghn_tune_trial) == 32  # 5 x 4 bytes, pad, double


def _build_raw(ghn, points=1, n=10, f=2, dtype=0, targets=2, task=0, widths=(0.5,), origin=None):
    L = ghn.lib()
    w = (ctypes.c_float * 32)(*widths) if widths is not None else None
    o = (ctypes.c_float * 32)(*origin) if origin is not None else None
    h = ctypes.c_void_p()
    pts = ctypes.c_void_p(points * 256) if points else None
    tg = ctypes.c_void_p(targets * 256) if targets else None
    code = L.ghn_build(pts, n, f, dtype, tg, task, w, len(widths) if widths else 1, o, None, ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("kw,code", [
    (dict(points=0), -1),
    (dict(targets=0), -1),
    (dict(n=0), -1),
    (dict(n=-5), -1),
    (dict(n=2 ** 31), -1),
    (dict(f=0), -1),
    (dict(f=33), -1),
    (dict(dtype=2), -1),
    (dict(task=5), -1),
    (dict(widths=(0.0,)), -1),
    (dict(widths=(-1.0,)), -1),
    (dict(widths=(float("nan"),)), -1),
    (dict(widths=(float("inf"),)), -1),
    (dict(widths=(0.5, 0.5, 0.5)), -1),       # n_width must be 1 or f
    (dict(origin=(float("nan"), 0.0)), -1),
])
def test_build_rejects_bad_arguments(ghn, kw, code):
    got, h = _build_raw(ghn, **kw)
    assert got == code
    assert not h.value
    assert ghn.ghn_last_error()


def test_predict_rejects_null_index(ghn):
    L = ghn.lib()
    code = L.ghn_predict(None, None, 1, 5, None, None, None, None, None, 0, None)
    assert code == -1
    assert "index" in ghn.ghn_last_error()


def test_destroy_null_is_noop(ghn):
    ghn.lib().ghn_destroy(None)


def test_load_rejects_bad_buffers(ghn):
    lib = ghn._lib
    out = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(b"not an index" * 40)
    assert lib.ghn_index_load(ctypes.cast(buf, ctypes.c_void_p), 12, None, ctypes.byref(out)) == -1
    assert lib.ghn_index_load(ctypes.cast(buf, ctypes.c_void_p), len(buf), None, ctypes.byref(out)) == -1
    assert not out.value
    assert lib.ghn_index_save_bytes(None) == 0
    assert lib.ghn_insert(None, None, 1, 0, None, None) == -1
