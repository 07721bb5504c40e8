"""Host-layer failure handling forced from the host (GHN_FAULT) and host logging
(GHN_LOG).  GHN_FAULT=alloc:N / launch:N makes the N-th device allocation or launch
check of the library fail; every such failure must return its status code with a
message, leak no device memory, leave no index behind (the handle stays NULL) and
leave the library working.  Leaks are found from GHN_LOG's allocation and release
lines (device free-memory figures are not exact: the runtime caches small blocks).  The kernels are untouched: an injected launch failure
only changes the status the host layer sees, after the launched work has finished."""
import ctypes
import os

import numpy as np
import pytest

from paper_2004_02290_amd import workloads as W

pytestmark = pytest.mark.gpu

NOMEM, HIP = -8, -7


@pytest.fixture(scope="module")
def ghn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_02290_amd import binding
    return binding


@pytest.fixture()
def fault_env():
    yield
    os.environ.pop("GHN_FAULT", None)
    os.environ.pop("GHN_LOG", None)


def _live(err):
    """Blocks the GHN_LOG lines show allocated and not released."""
    live = {}
    for line in err.splitlines():
        w = line.split()
        if line.startswith("ghn: alloc "):
            live[w[2]] = int(w[3])
        elif line.startswith("ghn: free "):
            live.pop(w[2], None)
    return live


def _small(ghn, lookup=None):
    import torch
    prob = W.make("clusters4d", n=20_000, m=2_000)
    pts = torch.from_numpy(prob.points).cuda()
    tg = torch.from_numpy(prob.targets).cuda()
    q = torch.from_numpy(prob.queries).cuda()
    return prob, pts, tg, q


def _raw_build(ghn, pts, tg, prob, lookup):
    """ghn_build_ex through the C ABI: (status, handle value)."""
    L = ghn._lib
    w, nw, o = ghn._widths(prob.cell_width, None)
    h = ctypes.c_void_p()
    opts = None if lookup is None else ctypes.byref(ghn.ghn_build_opts(int(lookup)))
    st = L.ghn_build_ex(ghn._ptr(pts), prob.n, prob.f, ghn._points_dtype(pts), ghn._ptr(tg), prob.task, w, nw, o, opts,
                        ghn._stream(None), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kind,lookup", [("alloc", None), ("alloc", 1), ("alloc", 2), ("launch", None), ("launch", 1),
                                         ("launch", 2)])
def test_build_fault_every_point(ghn, fault_env, kind, lookup, capfd):
    prob, pts, tg, q = _small(ghn)
    ref = ghn.Index(pts, tg, prob.task, prob.cell_width, lookup=lookup)
    want = ref.predict(q, 8)
    ref.close()
    want_code = NOMEM if kind == "alloc" else HIP
    os.environ["GHN_LOG"] = "1"
    capfd.readouterr()
    for n_at in range(1, 200):
        os.environ["GHN_FAULT"] = "%s:%d" % (kind, n_at)
        st, h = _raw_build(ghn, pts, tg, prob, lookup)
        if st == 0:
            break
        assert st == want_code, (n_at, st, ghn.ghn_last_error())
        assert h.value is None, "a failed build left an index behind"
        assert ghn.ghn_last_error() != ""
        err = capfd.readouterr().err
        assert "GHN_FAULT: " in err
        assert not _live(err), "a failed build at %s %d leaked %s" % (kind, n_at, _live(err))
    else:
        raise AssertionError("the build never got past the injected failures")
    assert n_at > 3, "too few %s points were reached" % kind
    os.environ.pop("GHN_FAULT")
    ghn.ghn_destroy(h)
    err = capfd.readouterr().err
    assert "ghn: build n=" in err and not _live(err), "the index did not release all its blocks"
    os.environ.pop("GHN_LOG")
    # the library still works and gives the same answers
    ix = ghn.Index(pts, tg, prob.task, prob.cell_width, lookup=lookup)
    got = ix.predict(q, 8)
    assert np.array_equal(got["idx"].cpu().numpy(), want["idx"].cpu().numpy())
    ix.close()


def test_predict_and_batch_launch_fault(ghn, fault_env):
    import torch
    prob, pts, tg, q = _small(ghn)
    ix = ghn.Index(pts, tg, prob.task, prob.cell_width)
    want = ix.predict(q, 8)
    for prec in (0, 1):
        os.environ["GHN_FAULT"] = "launch:1"
        with pytest.raises(ghn.GHNError) as ei:
            ix.predict(q, 8, prec=prec)
        assert ei.value.code == HIP
        os.environ.pop("GHN_FAULT")
        got = ix.predict(q, 8, prec=prec)
        assert np.array_equal(got["idx"].cpu().numpy(), want["idx"].cpu().numpy())
    oi = torch.empty((prob.m, 8), dtype=torch.int64, device="cuda")
    op = torch.empty(prob.m, dtype=torch.int32, device="cuda")
    items = [(ix.handle, q, 8, oi, op, None)]
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, 0)
    os.environ["GHN_FAULT"] = "launch:1"
    with pytest.raises(ghn.GHNError) as ei:
        ghn.ghn_predict_batched(batch)
    assert ei.value.code == HIP
    os.environ.pop("GHN_FAULT")
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    assert np.array_equal(oi.cpu().numpy(), want["idx"].cpu().numpy())
    ix.close()


def test_insert_and_measure_faults_leave_state(ghn, fault_env, capfd):
    import torch
    prob, pts, tg, q = _small(ghn)
    half = prob.n // 2
    # a successful insert and measurement first
    warm = ghn.Index(pts[:half].contiguous(), tg[:half].contiguous(), prob.task, prob.cell_width)
    ghn.ghn_insert(warm.handle, pts[half:].contiguous(), tg[half:].contiguous())
    warm.close()
    ghn.ghn_cell_measure(pts)
    ix = ghn.Index(pts[:half].contiguous(), tg[:half].contiguous(), prob.task, prob.cell_width)
    before = ix.predict(q, 8)["idx"].cpu().numpy()
    new_pts, new_tg = pts[half:].contiguous(), tg[half:].contiguous()
    os.environ["GHN_LOG"] = "1"
    capfd.readouterr()
    # an insert into a dense-table index allocates twice (its workspace, the new index's
    # block) and checks many launches
    for kind, code in (("alloc", NOMEM), ("launch", HIP)):
        for n_at in ((1, 2) if kind == "alloc" else (1, 2, 3, 6)):
            os.environ["GHN_FAULT"] = "%s:%d" % (kind, n_at)
            with pytest.raises(ghn.GHNError) as ei:
                ghn.ghn_insert(ix.handle, new_pts, new_tg)
            assert ei.value.code == code
            os.environ.pop("GHN_FAULT")
            err = capfd.readouterr().err
            assert not _live(err), "a failed insert at %s %d leaked %s" % (kind, n_at, _live(err))
            assert ghn.ghn_index_get_info(ix.handle).n == half
            assert np.array_equal(ix.predict(q, 8)["idx"].cpu().numpy(), before), "a failed insert changed the index"
    for kind, code in (("alloc", NOMEM), ("launch", HIP)):
        os.environ["GHN_FAULT"] = kind
        with pytest.raises(ghn.GHNError) as ei:
            ghn.ghn_cell_measure(pts)
        assert ei.value.code == code
        os.environ.pop("GHN_FAULT")
        err = capfd.readouterr().err
        assert not _live(err), "a failed measurement leaked %s" % _live(err)
    os.environ.pop("GHN_LOG")
    ix.close()


def test_log_lines(ghn, fault_env, capfd):
    prob, pts, tg, q = _small(ghn)
    os.environ["GHN_LOG"] = "1"
    ix = ghn.Index(pts, tg, prob.task, prob.cell_width)
    ix.predict(q, 8)
    with pytest.raises(ghn.GHNError):
        ix.predict(q, 0)
    os.environ["GHN_FAULT"] = "alloc"
    with pytest.raises(ghn.GHNError):
        ghn.Index(pts, tg, prob.task, prob.cell_width)
    os.environ.pop("GHN_LOG")
    os.environ.pop("GHN_FAULT")
    ix.predict(q, 8)
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("ghn: ")]
    assert any(l.startswith("ghn: build n=%d f=%d" % (prob.n, prob.f)) for l in lines), err
    assert sum(l.startswith("ghn: predict m=%d k=8" % prob.m) for l in lines) == 1, err
    assert any(l.startswith("ghn: error -1: ghn_predict: k=0") for l in lines), err
    assert any("GHN_FAULT: device allocation" in l for l in lines), err
    assert any(l.startswith("ghn: error -8:") for l in lines), err
    ix.close()
