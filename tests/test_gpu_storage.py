"""The build into caller-owned device memory (ghn_build_into): the index lives in a
torch tensor, the temporaries in another, and no device memory is allocated by the
library.  Results must equal the oracle's (EXACT: brute force; PAPER: the grid walk
with its stop layers) and those of the library-allocated index."""
import numpy as np
import pytest

import oracle
from paper_2004_02290_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ghn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_02290_amd import binding
    return binding


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _points(prob):
    import torch
    if prob.dtype == "bf16":
        return _dev(prob.points.view(np.int16)).view(torch.bfloat16)
    return _dev(prob.points)


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(got, want, what, layers=False):
    keys = ("idx", "d2", "pred") + (("stop_layer",) if layers else ())
    for key in keys:
        assert np.array_equal(got[key], want[key]), "%s: %s differs" % (what, key)


@pytest.mark.parametrize("name,kw,lookup", [
    ("clusters4d", dict(n=60_000, m=2_000), None),       # dense table
    ("skew8d", dict(n=80_000, m=600, seed=3), None),     # 8-D: the cell tree
    ("clusters4d", dict(n=40_000, m=1_500), 2),          # hash lookup
    ("bf16_16d", dict(n=30_000, m=300), None),           # bf16 points, 16-D
])
def test_build_into_torch_storage_matches_oracle(ghn, name, kw, lookup):
    import torch
    prob = W.make(name, **kw)
    pts, tg, q = _points(prob), _dev(prob.targets), _dev(prob.queries)
    ix = ghn.Index(pts, tg, prob.task, prob.cell_width, lookup=lookup, torch_storage=True)
    assert ix.storage is not None and ix.info.device_bytes <= ix.storage.numel()
    ref = ghn.Index(pts, tg, prob.task, prob.cell_width, lookup=lookup)
    assert ix.info.lookup == ref.info.lookup and ix.info.num_cells == ref.info.num_cells
    pf = prob.points_f32()
    bi, bd, bp = oracle.bruteforce(pf, prob.targets, prob.task, prob.queries, prob.k)
    want_paper = oracle.Grid(pf, prob.targets, prob.task, prob.cell_width).predict(prob.queries, prob.k,
                                                                                 oracle.STOP_PAPER)
    for prec in (ghn.GHN_PREC_FP32, ghn.GHN_PREC_BF16_MFMA):
        got = _host(ix.predict(q, prob.k, prec=prec, with_stats=True))
        _same(got, dict(idx=bi, d2=bd, pred=bp), "%s EXACT prec=%d" % (name, prec))
        _same(got, _host(ref.predict(q, prob.k, prec=prec, with_stats=True)), "%s vs library index" % name,
              layers=prec == ghn.GHN_PREC_FP32)
        got = _host(ix.predict(q, prob.k, stop=ghn.GHN_STOP_PAPER, prec=prec, with_stats=True))
        _same(got, want_paper, "%s PAPER prec=%d" % (name, prec), layers=True)
    # the index in torch storage also serves the persistent batched launch
    oi = torch.empty((prob.m, prob.k), dtype=torch.int64, device="cuda")
    op = torch.empty(prob.m, dtype=torch.int32 if prob.task == W.CLASSIFY else torch.float32, device="cuda")
    od = torch.empty((prob.m, prob.k), dtype=torch.float64, device="cuda")
    items = [(ix.handle, q, prob.k, oi, op, od)]
    bws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, bws)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    _same(dict(idx=oi.cpu().numpy(), d2=od.cpu().numpy(), pred=op.cpu().numpy()), dict(idx=bi, d2=bd, pred=bp),
          "%s batched from torch storage" % name)
    ghn.ghn_batch_destroy(batch)
    ix.close()
    ref.close()


def test_build_into_allocates_nothing(ghn):
    import torch
    prob = W.make("clusters4d", n=100_000, m=500)
    pts, tg = _points(prob), _dev(prob.targets)
    n, f = prob.points.shape
    ws = torch.empty(ghn.ghn_build_workspace_bytes(n, f), dtype=torch.uint8, device="cuda")
    nbytes = ghn.ghn_index_bytes_for(pts, prob.task, prob.cell_width, ws)
    assert nbytes <= ghn.ghn_index_bytes(n, f)
    storage = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = ghn.ghn_build_into(pts, tg, prob.task, prob.cell_width, storage, ws)  # loads the kernels
    ghn.ghn_destroy(h)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    h = ghn.ghn_build_into(pts, tg, prob.task, prob.cell_width, storage, ws)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    ghn.ghn_destroy(h)  # frees only the handle; the storage stays with torch
    del storage


def test_build_into_errors(ghn):
    import torch
    prob = W.make("blobs2d", m=10)
    pts, tg = _points(prob), _dev(prob.targets)
    n, f = prob.points.shape
    ws = torch.empty(ghn.ghn_build_workspace_bytes(n, f), dtype=torch.uint8, device="cuda")
    nbytes = ghn.ghn_index_bytes_for(pts, prob.task, prob.cell_width, ws)
    with pytest.raises(ghn.GHNError) as e:   # storage too small: refused after the cell-range pass
        ghn.ghn_build_into(pts, tg, prob.task, prob.cell_width, torch.empty(nbytes // 2, dtype=torch.uint8,
                                                                             device="cuda"), ws)
    assert e.value.code == -6
    with pytest.raises(ghn.GHNError) as e:   # workspace too small: refused before any launch
        ghn.ghn_build_into(pts, tg, prob.task, prob.cell_width, torch.empty(nbytes, dtype=torch.uint8, device="cuda"),
                           ws[: ws.numel() // 2])
    assert e.value.code == -6
    storage = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ghn.GHNError) as e:   # misaligned storage
        ghn.ghn_build_into(pts, tg, prob.task, prob.cell_width, storage[1:], ws)
    assert e.value.code == -1
    ix = ghn.Index(pts, tg, prob.task, prob.cell_width, torch_storage=True)
    with pytest.raises(ghn.GHNError) as e:   # insert into caller storage is refused
        ix.insert(pts[:10], tg[:10])
    assert e.value.code == -2
    ix.close()
