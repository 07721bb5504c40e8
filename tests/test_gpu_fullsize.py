"""Full-size parity on sampled outputs, in the launch configurations the benchmark
times.

Each workload is generated at its full size and the GPU answers every query; a
seeded sample of rows is then checked one by one against the oracle: brute-force
neighbours, distances and predictions (bit-identical), and for the per-query walks
the grid oracle's EXACT stop layers as well."""
import numpy as np
import pytest

import oracle
from paper_2004_02290_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32, BF16 = 0, 1
EXACT, PAPER = 0, 1


@pytest.fixture(scope="module")
def ghn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_02290_amd import binding
    return binding


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pts(prob):
    import torch
    if prob.dtype == "bf16":
        return _dev(prob.points.view(np.int16)).view(torch.bfloat16)
    return _dev(prob.points)


def _host(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(got, want, what, rows, keys=("idx", "d2", "pred")):
    for key in keys:
        g, w = got[key][rows], want[key]
        if not np.array_equal(g, w):
            bad = np.flatnonzero((g != w).reshape(g.shape[0], -1).any(axis=1))
            raise AssertionError("%s: %s differs on %d of %d sampled rows, first query %d: got %s want %s" % (
                what, key, bad.size, rows.size, rows[bad[0]], g[bad[0]], w[bad[0]]))


def _sample(m, count, seed):
    return np.sort(np.random.default_rng(seed).choice(m, min(m, count), replace=False))


def _brute(prob, rows):
    bi, bd, bp = oracle.bruteforce(prob.points_f32(), prob.targets, prob.task, prob.queries[rows], prob.k)
    return dict(idx=bi, d2=bd, pred=bp)


def _check(ghn, prob, ix, rows, brute, what, layers_from=None, **kw):
    got = _host(ix.predict(_dev(prob.queries), prob.k, with_stats=True, **kw))
    _same(got, brute, what, rows)
    if layers_from is not None:
        assert np.array_equal(got["stop_layer"][rows], layers_from), what + ": stop layers"
    return got


@pytest.mark.parametrize("width_scale", [1.0, 2.0 ** -0.5])
def test_skew8d_full_size(ghn, width_scale):
    """10M points, 1M queries: the calibrated width and the finer one the autotuner
    picks for the FP32 walk; FP32 in Morton order and in input order, the grouped bf16
    screen, and the persistent launch, all on the same sampled rows."""
    import torch
    prob = W.make("skew8d")
    width = np.float32(prob.cell_width * width_scale)
    ix = ghn.Index(_pts(prob), _dev(prob.targets), prob.task, float(width))
    assert ix.info.lookup == 1
    rows = _sample(prob.m, 160, 11)
    g = oracle.Grid(prob.points_f32(), prob.targets, prob.task, float(width))
    want = g.predict(prob.queries[rows], prob.k, oracle.STOP_EXACT)
    g.close()
    what = "skew8d w=%.6g" % width
    bw = _brute(prob, rows)
    a = _check(ghn, prob, ix, rows, bw, what + " FP32 sorted", layers_from=want["stop_layer"], prec=FP32)
    b = _check(ghn, prob, ix, rows, bw, what + " FP32 input order", layers_from=want["stop_layer"], prec=FP32,
               flags=ghn.GHN_FLAG_NO_SORT)
    assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(a["pred"], b["pred"])
    for levels in (0, 1):
        _check(ghn, prob, ix, rows, bw, what + " bf16 levels %d" % levels, layers_from=want["stop_layer"], prec=BF16,
               group_levels=levels)
    # persistent launch: every query, against the per-query kernel's answers
    oi = torch.empty((prob.m, prob.k), dtype=torch.int64, device="cuda")
    op = torch.empty(prob.m, dtype=torch.float32, device="cuda")
    od = torch.empty((prob.m, prob.k), dtype=torch.float64, device="cuda")
    q = _dev(prob.queries)  # the batch descriptor points at it until the launch has run
    items = [(ix.handle, q, prob.k, oi, op, od)]
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, EXACT)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    assert np.array_equal(oi.cpu().numpy(), b["idx"]) and np.array_equal(od.cpu().numpy(), b["d2"])
    assert np.array_equal(op.cpu().numpy(), b["pred"])
    ix.close()


@pytest.mark.parametrize("width_scale", [1.0, 2.0])
def test_bf16_16d_full_size(ghn, width_scale):
    """4M bf16 points in 16 dimensions, 500k queries, k = 32, at the calibrated width and
    the twice coarser one the autotuner picks: the FP32 tree walk (input and Morton
    order) and the grouped bf16 screen (default grouping and 2^2-cell groups), on
    sampled rows."""
    prob = W.make("bf16_16d")
    width = float(np.float32(prob.cell_width * width_scale))
    ix = ghn.Index(_pts(prob), _dev(prob.targets), prob.task, width)
    rows = _sample(prob.m, 200, 12)
    g = oracle.Grid(prob.points_f32(), prob.targets, prob.task, width)
    want = g.predict(prob.queries[rows], prob.k, oracle.STOP_EXACT)
    g.close()
    bw = _brute(prob, rows)
    what = "bf16_16d w=%.6g" % width
    _check(ghn, prob, ix, rows, bw, what + " FP32", layers_from=want["stop_layer"], prec=FP32,
           flags=ghn.GHN_FLAG_NO_SORT)
    _check(ghn, prob, ix, rows, bw, what + " FP32 sorted", layers_from=want["stop_layer"], prec=FP32)
    _check(ghn, prob, ix, rows, bw, what + " bf16", layers_from=want["stop_layer"], prec=BF16)
    _check(ghn, prob, ix, rows, bw, what + " bf16 levels 2", layers_from=want["stop_layer"], prec=BF16,
           group_levels=2)
    ix.close()


def test_multi3d_full_size_batched(ghn):
    """All 256 independent 3-D problems in one persistent launch (EXACT), as the
    benchmark times it; a few sampled queries of every problem against brute force."""
    import torch
    probs = W.make_multi3d()
    idxs, items, outs = [], [], []
    for p in probs:
        ix = ghn.Index(_dev(p.points), _dev(p.targets), p.task, p.cell_width)
        oi = torch.full((p.m, p.k), -7, dtype=torch.int64, device="cuda")
        op = torch.full((p.m,), -7, dtype=torch.int32, device="cuda")
        od = torch.zeros((p.m, p.k), dtype=torch.float64, device="cuda")
        idxs.append(ix)
        items.append((ix.handle, _dev(p.queries), p.k, oi, op, od))
        outs.append((oi, op, od))
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, EXACT)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    for i, (p, (oi, op, od)) in enumerate(zip(probs, outs)):
        rows = _sample(p.m, 6, 100 + i)
        bi, bd, bp = oracle.bruteforce(p.points, p.targets, p.task, p.queries[rows], p.k)
        got = dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy())
        _same(got, dict(idx=bi, d2=bd, pred=bp), "multi3d problem %d (n=%d, m=%d, k=%d)" % (i, p.n, p.m, p.k), rows)
    for ix in idxs:
        ix.close()
