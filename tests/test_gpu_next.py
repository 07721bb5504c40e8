"""GPU results against the CPU oracle for the paper's cell measurement rule (and
the wide cell codes its fine grids need), the median statistic and exhaustive
KNN, element by element (bit-identical)."""
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


def _pts(prob):
    import torch
    if prob.dtype == "bf16":
        return _dev(prob.points.view(np.int16)).view(torch.bfloat16)
    return _dev(prob.points)


def _host(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(got, want, what, keys=("idx", "d2", "pred")):
    for key in keys:
        g, w = got[key], want[key]
        if not np.array_equal(g, w):
            bad = np.flatnonzero((g != w).reshape(g.shape[0], -1).any(axis=1))
            raise AssertionError("%s: %s differs on %d rows, first %d: got %s want %s" % (
                what, key, bad.size, bad[0], g[bad[0]], w[bad[0]]))


# ------------------------------------------------------------------------- cell measurements
def _measure_cases():
    rng = np.random.default_rng(21)
    yield "counterexample", np.array([[0.28], [0.485], [0.75], [0.981]], np.float32)
    yield "blobs2d", W.make("blobs2d", n=3000, m=1).points
    yield "uniform3", rng.random((2500, 3), dtype=np.float32)
    yield "lattice", W.lattice_problem(2000, 1, 2, 1).points
    yield "negative", (rng.normal(0, 3, (1500, 4)) ** 3).astype(np.float32)
    yield "constant", np.concatenate([np.full((500, 1), 7.5, np.float32), rng.random((500, 1), dtype=np.float32)], 1)
    yield "single", np.array([[1.0, -2.0]], np.float32)


@pytest.mark.parametrize("case", range(7))
def test_cell_measure_matches_oracle(ghn, case):
    name, x = list(_measure_cases())[case]
    w, o, s = ghn.ghn_cell_measure(_dev(x))
    ww, wo, ws = oracle.cell_measure(x)
    assert np.array_equal(s, ws), (name, s, ws)
    assert np.array_equal(w, ww), (name, w, ww)
    assert np.array_equal(o, wo), (name, o, wo)


def test_cell_measure_bf16_points(ghn):
    prob = W.make("bf16_16d", n=1500, m=1)
    w, o, s = ghn.ghn_cell_measure(_pts(prob))
    ww, wo, ws = oracle.cell_measure(prob.points_f32())
    assert np.array_equal(s, ws) and np.array_equal(w, ww) and np.array_equal(o, wo)


def _split_of(x, o, w, s):
    v = x.astype(np.float64) - float(o)
    q = np.floor(v / float(w))
    q = np.where(q * float(w) > v, q - 1, q)
    q = np.where((q + 1) * float(w) <= v, q + 1, q)
    return np.minimum(q, s - 1).astype(np.int64)


def test_cell_measure_full_size_properties(ghn):
    # 1M points: the oracle's search over every split count is too slow here, so the
    # defining property is checked: s splits all hold points, the next counts do not
    prob = W.make("clusters4d")
    w, o, s = ghn.ghn_cell_measure(_dev(prob.points))
    for j in range(prob.f):
        col = prob.points[:, j]
        assert o[j] == col.min()
        assert np.unique(_split_of(col, o[j], w[j], s[j])).size == s[j]
        rng_ = float(col.max()) - float(col.min())
        for s2 in range(int(s[j]) + 1, int(s[j]) + 25):
            w2 = np.float32(rng_ / s2)
            assert np.unique(_split_of(col, o[j], w2, s2)).size < s2, (j, s2)


def test_paper_widths_build_and_predict(ghn):
    # the paper's own configuration: measured widths and origin, PAPER and EXACT rules
    prob = W.make("blobs2d")
    w, o, s = ghn.ghn_cell_measure(_dev(prob.points))
    ix = ghn.Index(_dev(prob.points), _dev(prob.targets), prob.task, w, o)
    q = _dev(prob.queries)
    g = oracle.Grid(prob.points, prob.targets, prob.task, w, o)
    got = _host(ix.predict(q, prob.k, stop=ghn.GHN_STOP_PAPER, with_stats=True))
    want = g.predict(prob.queries, prob.k, oracle.STOP_PAPER)
    _same(got, want, "PAPER with measured widths")
    assert np.array_equal(got["stop_layer"], want["stop_layer"])
    got = _host(ix.predict(q, prob.k, stop=ghn.GHN_STOP_EXACT))
    bi, bd, bp = oracle.bruteforce(prob.points, prob.targets, prob.task, prob.queries, prob.k)
    _same(got, dict(idx=bi, d2=bd, pred=bp), "EXACT with measured widths")


@pytest.mark.parametrize("f,n,m,width", [(8, 6000, 400, 0.0025), (16, 4000, 300, 0.01), (32, 1500, 200, 0.05)])
def test_wide_cell_codes(ghn, f, n, m, width):
    # fine grids (such as the paper's rule gives on clustered data) whose Morton codes need
    # more than 64 bits: multi-word sort on build, top-64-bit keys for query order and groups
    rng = np.random.default_rng(f)
    c = rng.random((4, f))
    pts = (c[rng.integers(0, 4, n)] + rng.normal(0, 0.01, (n, f))).astype(np.float32)
    qs = (c[rng.integers(0, 4, m)] + rng.normal(0, 0.02, (m, f))).astype(np.float32)
    lab = rng.integers(0, 5, n).astype(np.int32)
    cid = np.floor(pts.astype(np.float64) / width).astype(np.int64)
    bits = sum(int(x).bit_length() for x in cid.max(0) - cid.min(0))
    assert bits > 64, bits
    ix = ghn.Index(_dev(pts), _dev(lab), 0, width)
    assert ix.info.lookup == 1
    k = 7
    bi, bd, bp = oracle.bruteforce(pts, lab, 0, qs, k)
    want_paper = oracle.Grid(pts, lab, 0, width).predict(qs, k, oracle.STOP_PAPER)
    for prec in (0, 1):
        got = _host(ix.predict(_dev(qs), k, prec=prec))
        _same(got, dict(idx=bi, d2=bd, pred=bp), "wide f=%d EXACT prec=%d" % (f, prec))
        got = _host(ix.predict(_dev(qs), k, stop=ghn.GHN_STOP_PAPER, prec=prec, with_stats=True))
        _same(got, want_paper, "wide f=%d PAPER prec=%d" % (f, prec))
        assert np.array_equal(got["stop_layer"], want_paper["stop_layer"])


def test_cell_measure_errors(ghn):
    x = np.array([[0.0, 1.0], [np.nan, 2.0]], np.float32)
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_cell_measure(_dev(x))
    assert e.value.code == -4


# ------------------------------------------------------------------------------- median
@pytest.mark.parametrize("prec", [0, 1])
def test_median_regression(ghn, prec):
    prob = W.make("skew8d", n=40_000, m=1_500)
    ix = ghn.Index(_dev(prob.points), _dev(prob.targets), prob.task, prob.cell_width)
    q = _dev(prob.queries)
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        got = _host(ix.predict(q, prob.k, stop=stop, prec=prec, flags=ghn.GHN_FLAG_MEDIAN, with_stats=True))
        if stop == ghn.GHN_STOP_EXACT:
            bi, bd, bp = oracle.bruteforce(prob.points, prob.targets, oracle.REGRESS_MEDIAN, prob.queries, prob.k)
            want = dict(idx=bi, d2=bd, pred=bp)
        else:
            want = oracle.Grid(prob.points, prob.targets, oracle.REGRESS_MEDIAN, prob.cell_width).predict(
                prob.queries, prob.k, oracle.STOP_PAPER)
        _same(got, want, "median stop=%d prec=%d" % (stop, prec))


def test_median_ties_and_even_k(ghn):
    base = W.lattice_problem(3000, 400, 3, 1, task=W.REGRESS)
    y = np.round(base.targets * 2).astype(np.float32) / 2   # many equal targets
    for k in (1, 2, 5, 8, 33, 64):
        ix = ghn.Index(_dev(base.points), _dev(y), W.REGRESS, base.cell_width)
        for prec in (0, 1):
            got = _host(ix.predict(_dev(base.queries), k, prec=prec, flags=ghn.GHN_FLAG_MEDIAN))
            bi, bd, bp = oracle.bruteforce(base.points, y, oracle.REGRESS_MEDIAN, base.queries, k)
            _same(got, dict(idx=bi, d2=bd, pred=bp), "median k=%d prec=%d" % (k, prec))


def test_median_batched_and_errors(ghn):
    import torch
    prob = W.make("skew8d", n=20_000, m=600)
    ix = ghn.Index(_dev(prob.points), _dev(prob.targets), prob.task, prob.cell_width)
    q = _dev(prob.queries)
    oi = torch.empty((prob.m, prob.k), dtype=torch.int64, device="cuda")
    op = torch.empty(prob.m, dtype=torch.float32, device="cuda")
    items = [(ix.handle, q, prob.k, oi, op, None)]
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, flags=ghn.GHN_FLAG_MEDIAN), dtype=torch.uint8, device="cuda")
    b = ghn.ghn_batch_prepare(items, ws, flags=ghn.GHN_FLAG_MEDIAN)
    ghn.ghn_predict_batched(b)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(b)
    _, _, bp = oracle.bruteforce(prob.points, prob.targets, oracle.REGRESS_MEDIAN, prob.queries, prob.k)
    assert np.array_equal(op.cpu().numpy(), bp)
    c = W.make("blobs2d", n=2000, m=10)
    cix = ghn.Index(_dev(c.points), _dev(c.targets), c.task, c.cell_width)
    with pytest.raises(ghn.GHNError) as e:
        cix.predict(_dev(c.queries), c.k, flags=ghn.GHN_FLAG_MEDIAN)
    assert e.value.code == -1


# ------------------------------------------------------------------------------ brute force
@pytest.mark.parametrize("name,n,m,k", [("blobs2d", None, None, 5), ("clusters4d", 50_000, 700, 10),
                                        ("skew8d", 30_000, 500, 16), ("bf16_16d", 20_000, 300, 32)])
def test_bruteforce_matches_oracle(ghn, name, n, m, k):
    prob = W.make(name, n=n, m=m)
    ix = ghn.Index(_pts(prob), _dev(prob.targets), prob.task, prob.cell_width)
    got = _host(ix.bruteforce(_dev(prob.queries), k, with_stats=True))
    bi, bd, bp = oracle.bruteforce(prob.points_f32(), prob.targets, prob.task, prob.queries, k)
    _same(got, dict(idx=bi, d2=bd, pred=bp), name + " bruteforce")
    assert (got["cands"] == prob.n).all()


def test_bruteforce_ties_k_range_and_median(ghn):
    base = W.lattice_problem(1500, 300, 2, 1)
    ix = ghn.Index(_dev(base.points), _dev(base.targets), base.task, base.cell_width)
    for k in (1, 3, 16, 17, 40, 64):
        got = _host(ix.bruteforce(_dev(base.queries), k))
        bi, bd, bp = oracle.bruteforce(base.points, base.targets, base.task, base.queries, k)
        _same(got, dict(idx=bi, d2=bd, pred=bp), "lattice bruteforce k=%d" % k)
    r = W.lattice_problem(1500, 300, 4, 1, task=W.REGRESS)
    rix = ghn.Index(_dev(r.points), _dev(r.targets), r.task, r.cell_width)
    got = _host(rix.bruteforce(_dev(r.queries), 12, flags=ghn.GHN_FLAG_MEDIAN))
    bi, bd, bp = oracle.bruteforce(r.points, r.targets, oracle.REGRESS_MEDIAN, r.queries, 12)
    _same(got, dict(idx=bi, d2=bd, pred=bp), "lattice bruteforce median")


# ----------------------------------------------------------------------- save / load / insert
def _all_forms(ghn, ix, q, k):
    out = {}
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        for prec in (0, 1):
            out[(stop, prec)] = _host(ix.predict(q, k, stop=stop, prec=prec, with_stats=True))
    return out


@pytest.mark.parametrize("name,n,m", [("clusters4d", 40_000, 800), ("bf16_16d", 20_000, 300)])
def test_save_load_roundtrip(ghn, name, n, m):
    prob = W.make(name, n=n, m=m)
    ix = ghn.Index(_pts(prob), _dev(prob.targets), prob.task, prob.cell_width)
    data = ix.save()
    back = ghn.Index.load(data)
    for key in ("n", "f", "dtype", "task", "lookup", "num_cells"):
        assert getattr(back.info, key) == getattr(ix.info, key), key
    q = _dev(prob.queries)
    a, b = _all_forms(ghn, ix, q, prob.k), _all_forms(ghn, back, q, prob.k)
    for key in a:
        _same(b[key], a[key], "%s loaded %s" % (name, key), keys=("idx", "d2", "pred", "stop_layer"))


def test_insert_matches_fresh_build(ghn):
    import torch
    prob = W.make("clusters4d", n=30_000, m=600)
    pts, tgt = prob.points, prob.targets
    # the last chunk lies partly outside the first chunk's box, so the box grows
    extra = (pts[:2000] * 1.7 - 0.3).astype(np.float32)
    all_pts = np.concatenate([pts, extra])
    all_tgt = np.concatenate([tgt, tgt[:2000]])
    cut = [0, 18_000, 27_000, all_pts.shape[0]]
    ix = ghn.Index(_dev(all_pts[:cut[1]]), _dev(all_tgt[:cut[1]]), prob.task, prob.cell_width)
    for a, b in zip(cut[1:-1], cut[2:]):
        ix.insert(_dev(all_pts[a:b]), _dev(all_tgt[a:b]))
    assert ix.info.n == all_pts.shape[0]
    fresh = ghn.Index(_dev(all_pts), _dev(all_tgt), prob.task, prob.cell_width)
    assert ix.info.num_cells == fresh.info.num_cells and ix.info.lookup == fresh.info.lookup
    q = _dev(prob.queries)
    a, b = _all_forms(ghn, ix, q, prob.k), _all_forms(ghn, fresh, q, prob.k)
    for key in a:
        _same(a[key], b[key], "inserted vs fresh %s" % (key,), keys=("idx", "d2", "pred", "stop_layer"))
    bi, bd, bp = oracle.bruteforce(all_pts, all_tgt, prob.task, prob.queries, prob.k)
    _same(a[(ghn.GHN_STOP_EXACT, 0)], dict(idx=bi, d2=bd, pred=bp), "inserted EXACT vs oracle")
    want = oracle.Grid(all_pts, all_tgt, prob.task, prob.cell_width).predict(prob.queries, prob.k, oracle.STOP_PAPER)
    _same(a[(ghn.GHN_STOP_PAPER, 0)], want, "inserted PAPER vs oracle", keys=("idx", "d2", "pred", "stop_layer"))
    with pytest.raises(ValueError):
        ix.insert(_dev(all_pts[:5, :3]), _dev(all_tgt[:5]))


@pytest.mark.parametrize("lookup", [None, 2, 1])
def test_insert_merge_paths(ghn, lookup, capfd, monkeypatch):
    """Dense-table and hash indexes take the new points by a merge into their cell order
    (Algorithm 1's append; only the new points are sorted), a tree index by a rebuild;
    either way the index equals a build of all the points: the same cells, the same
    point order, and the same answers as the oracle."""
    prob = W.make("clusters4d", n=40_000, m=500)
    pts, tgt = prob.points, prob.targets
    # one chunk grows the box below the occupied cells, one lies inside it
    extra = (pts[:3000] * 1.5 - 0.4).astype(np.float32)
    all_pts = np.concatenate([pts, extra])
    all_tgt = np.concatenate([tgt, tgt[:3000] + 1])
    cut = [0, 25_000, 40_000, all_pts.shape[0]]
    ix = ghn.Index(_dev(all_pts[:cut[1]]), _dev(all_tgt[:cut[1]]), prob.task, prob.cell_width, lookup=lookup)
    monkeypatch.setenv("GHN_LOG", "1")
    capfd.readouterr()
    for a, b in zip(cut[1:-1], cut[2:]):
        ix.insert(_dev(all_pts[a:b]), _dev(all_tgt[a:b]))
    log = capfd.readouterr().err
    monkeypatch.delenv("GHN_LOG")
    how = "rebuilt from all points" if lookup == 1 else "merged into the cell order"
    assert log.count(how) == 2, log[-2000:]
    fresh = ghn.Index(_dev(all_pts), _dev(all_tgt), prob.task, prob.cell_width, lookup=lookup)
    assert ix.info.lookup == fresh.info.lookup and ix.info.num_cells == fresh.info.num_cells
    for x, y in zip(ghn.ghn_index_cells(ix.handle), ghn.ghn_index_cells(fresh.handle)):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    q = _dev(prob.queries)
    got = _all_forms(ghn, ix, q, prob.k)
    bi, bd, bp = oracle.bruteforce(all_pts, all_tgt, prob.task, prob.queries, prob.k)
    _same(got[(ghn.GHN_STOP_EXACT, 0)], dict(idx=bi, d2=bd, pred=bp), "inserted EXACT vs oracle")
    want = oracle.Grid(all_pts, all_tgt, prob.task, prob.cell_width).predict(prob.queries, prob.k, oracle.STOP_PAPER)
    _same(got[(ghn.GHN_STOP_PAPER, 0)], want, "inserted PAPER vs oracle", keys=("idx", "d2", "pred", "stop_layer"))
    ix.close()
    fresh.close()


def test_insert_bf16_and_bad_load(ghn):
    import torch
    prob = W.make("bf16_16d", n=12_000, m=200)
    half = prob.n // 2
    ix = ghn.Index(_dev(prob.points[:half].view(np.int16)).view(torch.bfloat16), _dev(prob.targets[:half]),
                   prob.task, prob.cell_width)
    ix.insert(_dev(prob.points[half:].view(np.int16)).view(torch.bfloat16), _dev(prob.targets[half:]))
    assert ix.info.dtype == ghn.GHN_BF16
    got = _host(ix.predict(_dev(prob.queries), prob.k))
    bi, bd, bp = oracle.bruteforce(prob.points_f32(), prob.targets, prob.task, prob.queries, prob.k)
    _same(got, dict(idx=bi, d2=bd, pred=bp), "bf16 insert")
    data = bytearray(ix.save())
    data[0] ^= 0xFF
    with pytest.raises(ghn.GHNError) as e:
        ghn.Index.load(bytes(data))
    assert e.value.code == -1


# ------------------------------------------------------------------------------ graph capture
def test_predict_graph_replay(ghn):
    # ghn_predict launches only kernels (no memset nodes): the FP32 walk with its query
    # sort and the grouped bf16 screen are captured once and replayed
    import torch
    prob = W.make("clusters4d", n=40_000, m=5_000)
    ix = ghn.Index(_dev(prob.points), _dev(prob.targets), prob.task, prob.cell_width)
    q = _dev(prob.queries)
    m, k = prob.m, prob.k
    runs = []
    for prec in (ghn.GHN_PREC_FP32, ghn.GHN_PREC_BF16_MFMA):
        oi = torch.empty((m, k), dtype=torch.int64, device="cuda")
        op = torch.empty(m, dtype=torch.int32, device="cuda")
        od = torch.empty((m, k), dtype=torch.float64, device="cuda")
        nb = ghn.ghn_predict_workspace_bytes(ix.handle, m, k, ghn.GHN_STOP_EXACT, prec, 0)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
        runs.append((prec, oi, op, od, ws))
    want = {}
    for prec, oi, op, od, ws in runs:
        ghn.ghn_predict(ix.handle, q, k, oi, op, od, ghn.GHN_STOP_EXACT, prec, 0, ws=ws)
        torch.cuda.synchronize()
        want[prec] = (oi.clone(), op.clone(), od.clone())
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for prec, oi, op, od, ws in runs:
                ghn.ghn_predict(ix.handle, q, k, oi, op, od, ghn.GHN_STOP_EXACT, prec, 0, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for prec, oi, op, od, ws in runs:      # eager work between replays
            oi.fill_(-1); op.fill_(-1); od.zero_(); ws.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for prec, oi, op, od, ws in runs:
            wi, wp, wd = want[prec]
            assert torch.equal(oi, wi) and torch.equal(op, wp) and torch.equal(od, wd), (rep, prec)
    bi, bd, bp = oracle.bruteforce(prob.points, prob.targets, prob.task, prob.queries, k)
    assert np.array_equal(want[ghn.GHN_PREC_FP32][0].cpu().numpy(), bi)


# ------------------------------------------------------------------- screen error and re-rank band
BOUND_REL = 2.0 ** -13.8   # proven bound of |s - d| / (|q'|^2 + |x'|^2) for the bf16 screen


def _offset_problem(seed, f, lo, hi, n=20_000, m=256):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(lo, hi, (n, f)).astype(np.float32)
    qs = rng.uniform(lo, hi, (m, f)).astype(np.float32)
    lab = rng.integers(0, 3, n).astype(np.int32)
    return W.Problem("offset", pts, lab, qs, 8, W.CLASSIFY, float(np.float32((hi - lo) / 30.0)))


@pytest.mark.parametrize("case", ["clusters4d", "bf16_16d", "skew8d", "far", "wide"])
def test_screen_error_within_bound(ghn, case):
    if case == "far":
        prob = _offset_problem(1, 4, 1000.0, 1000.5)     # large coordinates, small spread
    elif case == "wide":
        prob = _offset_problem(2, 3, -1000.0, 1000.0)    # large spread
    else:
        prob = W.make(case, n=30_000, m=512)
    ix = ghn.Index(_pts(prob), _dev(prob.targets), prob.task, prob.cell_width)
    ea, er = ghn.ghn_screen_error(ix.handle, _dev(prob.queries), sample=4096)
    ea, er = ea.cpu().numpy(), er.cpu().numpy()
    assert np.isfinite(er).all() and er.max() < BOUND_REL, (case, er.max(), BOUND_REL)
    # the exact re-rank: at least k candidates are re-scored in FP64, never more than scored
    for prec in (0, 1):
        got = _host(ix.predict(_dev(prob.queries), prob.k, prec=prec, with_stats=True))
        assert (got["rerank"] >= prob.k).all() and (got["rerank"] <= got["cands"]).all(), (case, prec)
