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


def test_struct_sizes_match_header(ghn, tmp_path):
    """The binding's ctypes structures have the size and field offsets the C compiler
    gives the header's structures."""
    import subprocess
    structs = {"ghn_index_info": ghn.ghn_index_info, "ghn_predict_opts": ghn.ghn_predict_opts,
               "ghn_batch_item": ghn.ghn_batch_item, "ghn_tune_trial": ghn.ghn_tune_trial,
               "ghn_build_opts": ghn.ghn_build_opts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ghn.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines.append("return 0; }")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got["%s.%s" % (name, field)]) == getattr(cls, field).offset, (name, field)


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
