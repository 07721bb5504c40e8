"""GPU (HIP, gfx950) results against the CPU oracle, element by element.

Neighbour ids, FP64 distances, labels and regression means must be bit-identical:
  * EXACT stop rule  -> brute-force KNN (the plain definition);
  * PAPER stop rule  -> the oracle's grid walk, including the layer it stopped at.
"""
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


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _index(ghn, prob, widths=None, origin=None, lookup=None):
    import torch
    if prob.dtype == "bf16":
        pts = _dev(prob.points.view(np.int16)).view(torch.bfloat16)
    else:
        pts = _dev(prob.points)
    return ghn.Index(pts, _dev(prob.targets), prob.task, prob.cell_width if widths is None else widths, origin,
                     lookup=lookup)


def _run(ghn, ix, queries, k, stop, **kw):
    import torch
    out = ix.predict(_dev(queries), k, stop=stop, with_stats=True, **kw)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def _assert_same(got, want, what, check_layers=False):
    for key in ("idx", "d2", "pred"):
        g, w = got[key], want[key]
        if not np.array_equal(g, w):
            bad = np.flatnonzero((g != w).reshape(g.shape[0], -1).any(axis=1))
            raise AssertionError("%s: %s differs on %d rows, first %d: got %s want %s" % (
                what, key, bad.size, bad[0], g[bad[0]], w[bad[0]]))
    if check_layers:
        assert np.array_equal(got["stop_layer"], want["stop_layer"]), what


def _check_exact(ghn, prob, sample=None, seed=0, **kw):
    ix = _index(ghn, prob, **{k: v for k, v in kw.items() if k in ("widths", "origin", "lookup")})
    flags = kw.get("flags", 0)
    got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT, flags=flags)
    rows = np.arange(prob.m)
    if sample is not None and sample < prob.m:
        rows = np.sort(np.random.default_rng(seed).choice(prob.m, sample, replace=False))
    bi, bd, bp = oracle.bruteforce(prob.points_f32(), prob.targets, prob.task, prob.queries[rows], prob.k)
    _assert_same({k: v[rows] for k, v in got.items()}, dict(idx=bi, d2=bd, pred=bp), prob.name + " EXACT")
    return ix, got


def _check_paper(ghn, prob, sample=None, seed=1, widths=None, origin=None, flags=0, lookup=None):
    ix = _index(ghn, prob, widths, origin, lookup)
    got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_PAPER, flags=flags)
    rows = np.arange(prob.m)
    if sample is not None and sample < prob.m:
        rows = np.sort(np.random.default_rng(seed).choice(prob.m, sample, replace=False))
    g = oracle.Grid(prob.points_f32(), prob.targets, prob.task, prob.cell_width if widths is None else widths,
                    origin)
    want = g.predict(prob.queries[rows], prob.k, oracle.STOP_PAPER)
    _assert_same({k: v[rows] for k, v in got.items()}, want, prob.name + " PAPER", check_layers=True)
    return got


# ---------------------------------------------------------------------------------- workloads
def test_blobs2d_full_exact_and_paper(ghn):
    prob = W.make("blobs2d")
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_clusters4d_small_exact_and_paper(ghn):
    prob = W.make("clusters4d", n=60_000, m=3_001)
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_clusters4d_full_size_sampled(ghn):
    prob = W.make("clusters4d")
    _check_exact(ghn, prob, sample=1500)
    _check_paper(ghn, prob, sample=3000)


def test_exact_stop_layer_matches_oracle(ghn):
    prob = W.make("clusters4d", n=40_000, m=997)
    ix = _index(ghn, prob)
    got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT)
    want = oracle.Grid(prob.points, prob.targets, prob.task, prob.cell_width).predict(
        prob.queries, prob.k, oracle.STOP_EXACT)
    _assert_same(got, want, "EXACT vs grid oracle", check_layers=True)


def test_no_prune_same_result(ghn):
    prob = W.make("clusters4d", n=20_000, m=500)
    ix = _index(ghn, prob)
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        a = _run(ghn, ix, prob.queries, prob.k, stop)
        b = _run(ghn, ix, prob.queries, prob.k, stop, flags=ghn.GHN_FLAG_NO_PRUNE)
        _assert_same(a, b, "prune vs no-prune", check_layers=True)
        assert (b["cands"] >= a["cands"]).all()


def test_query_sort_same_result_and_workspace(ghn):
    import torch
    prob = W.make("clusters4d", n=50_000, m=9_000)
    ix = _index(ghn, prob)
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        a = _run(ghn, ix, prob.queries, prob.k, stop)
        b = _run(ghn, ix, prob.queries, prob.k, stop, flags=ghn.GHN_FLAG_NO_SORT)
        _assert_same(a, b, "sorted vs input order", check_layers=True)
        assert np.array_equal(a["cands"], b["cands"])
    assert ghn.ghn_predict_workspace_bytes(ix.handle, prob.m, prob.k) > 0
    assert ghn.ghn_predict_workspace_bytes(ix.handle, prob.m, prob.k, flags=ghn.GHN_FLAG_NO_SORT) == 0
    q = _dev(prob.queries)
    idx = torch.empty((prob.m, prob.k), dtype=torch.int64, device="cuda")
    pred = torch.empty(prob.m, dtype=torch.int32, device="cuda")
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_predict(ix.handle, q, prob.k, idx, pred)
    assert e.value.code == -6
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_predict(ix.handle, q, prob.k, idx, pred, ws=small)
    assert e.value.code == -6
    # an explicit order from ghn_query_order: a permutation, same results, no workspace
    order = torch.empty(prob.m, dtype=torch.int32, device="cuda")
    ows = torch.empty(ghn.ghn_query_order_workspace_bytes(prob.m), dtype=torch.uint8, device="cuda")
    ghn.ghn_query_order(ix.handle, q, order, ows)
    torch.cuda.synchronize()
    assert np.array_equal(np.sort(order.cpu().numpy()), np.arange(prob.m))
    d2 = torch.empty((prob.m, prob.k), dtype=torch.float64, device="cuda")
    ghn.ghn_predict(ix.handle, q, prob.k, idx, pred, d2, order=order)
    torch.cuda.synchronize()
    want = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT)
    assert np.array_equal(idx.cpu().numpy(), want["idx"]) and np.array_equal(d2.cpu().numpy(), want["d2"])


def test_deterministic(ghn):
    prob = W.make("clusters4d", n=30_000, m=800)
    ix = _index(ghn, prob)
    a = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_PAPER)
    b = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_PAPER)
    for key in a:
        assert np.array_equal(a[key], b[key])


# ---------------------------------------------------------------------------------- shapes, dims
@pytest.mark.parametrize("f", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dims_uniform(ghn, f):
    n = {1: 3000, 2: 3000, 3: 5000, 4: 6000, 5: 6000, 6: 8000, 7: 8000, 8: 8000}[f]
    width = {1: 0.003, 2: 0.05, 3: 0.1, 4: 0.2, 5: 0.3, 6: 0.34, 7: 0.5, 8: 0.5}[f]
    prob = W.uniform_problem(n=n, m=333, f=f, k=7, seed=f, width=width, q_lo=-0.3, q_hi=1.3)
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


@pytest.mark.parametrize("k", [1, 2, 13, 33, 64])
def test_k_values(ghn, k):
    prob = W.uniform_problem(n=4000, m=257, f=3, k=k, seed=100 + k, width=0.08)
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_k_equals_n(ghn):
    prob = W.uniform_problem(n=40, m=65, f=2, k=40, seed=9, width=0.3, q_lo=-2.0, q_hi=3.0)
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_lattice_ties_and_duplicates(ghn):
    for f in (2, 3):
        prob = W.lattice_problem(n=3000, m=300, f=f, k=12, seed=f)
        _check_exact(ghn, prob)
        _check_paper(ghn, prob)
        reg = W.lattice_problem(n=3000, m=300, f=f, k=12, seed=f, task=W.REGRESS)
        _check_exact(ghn, reg)


def test_regression_mean(ghn):
    prob = W.uniform_problem(n=20000, m=1000, f=3, k=16, seed=4, task=W.REGRESS, width=0.05)
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_per_dim_widths_and_origin(ghn):
    prob = W.uniform_problem(n=8000, m=400, f=3, k=9, seed=21, lo=-2.0, hi=2.0, q_lo=-3.0, q_hi=3.0)
    widths = np.array([0.31, 0.07, 0.19], np.float32)
    origin = np.array([-0.123, 0.05, 1.7], np.float32)
    _check_exact(ghn, prob, widths=widths, origin=origin)
    _check_paper(ghn, prob, widths=widths, origin=origin)


def test_far_queries(ghn):
    prob = W.uniform_problem(n=5000, m=200, f=3, k=5, seed=5, width=0.1)
    prob.queries[:50] *= 1e3
    prob.queries[50:100] -= 37.0
    prob.queries[100:110, 0] = 1e7
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_queries_on_points(ghn):
    prob = W.make("clusters4d", n=20000, m=10)
    prob.queries = prob.points[::37].copy()
    _check_exact(ghn, prob)
    _check_paper(ghn, prob)


def test_single_point_and_single_cell(ghn):
    p = W.uniform_problem(n=1, m=70, f=2, k=1, seed=3, width=0.5, q_lo=-5, q_hi=5)
    _check_exact(ghn, p)
    _check_paper(ghn, p)
    p = W.uniform_problem(n=500, m=70, f=3, k=20, seed=3, width=100.0)
    _check_exact(ghn, p)
    _check_paper(ghn, p)


# ---------------------------------------------------------------------------------- errors
def test_nonfinite_query_gets_sentinels(ghn):
    prob = W.uniform_problem(n=1000, m=8, f=2, k=3, seed=1, width=0.1)
    prob.queries[3, 1] = np.nan
    prob.queries[5, 0] = np.inf
    ix = _index(ghn, prob)
    got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT)
    for r in (3, 5):
        assert (got["idx"][r] == -1).all() and np.isnan(got["d2"][r]).all() and got["pred"][r] == -1
    ok = [0, 1, 2, 4, 6, 7]
    bi, bd, bp = oracle.bruteforce(prob.points, prob.targets, prob.task, prob.queries[ok], prob.k)
    assert np.array_equal(got["idx"][ok], bi) and np.array_equal(got["d2"][ok], bd)


def test_build_errors(ghn):
    pts = np.random.default_rng(0).random((100, 2)).astype(np.float32)
    lab = np.zeros(100, np.int32)
    bad = pts.copy()
    bad[7, 1] = np.nan
    with pytest.raises(ghn.GHNError) as e:
        ghn.Index(_dev(bad), _dev(lab), 0, 0.1)
    assert e.value.code == -4
    big = pts.copy()
    big[3, 0] = 1e30
    with pytest.raises(ghn.GHNError) as e:
        ghn.Index(_dev(big), _dev(lab), 0, 0.1)
    assert e.value.code == -5
    spread = pts.copy()
    spread[:, 0] *= 1e5
    spread[:, 1] *= 1e5
    with pytest.raises(ghn.GHNError) as e:
        ghn.Index(_dev(spread), _dev(lab), 0, 0.01, lookup=0)
    assert e.value.code == -2
    ix = ghn.Index(_dev(spread), _dev(lab), 0, 0.01)  # automatic choice falls back to the tree
    assert ix.info.lookup == 1
    wide = np.random.default_rng(1).random((200, 32)).astype(np.float32)  # 32 dims x 4 bits: 128-bit codes
    assert ghn.Index(_dev(wide), _dev(np.zeros(200, np.int32)), 0, 0.1).info.lookup == 1
    with pytest.raises(ghn.GHNError) as e:
        ghn.Index(_dev(pts), _dev(lab), 0, 0.1, lookup=7)
    assert e.value.code == -1


def test_predict_errors_and_empty(ghn):
    import torch
    prob = W.uniform_problem(n=50, m=4, f=2, k=3, seed=1, width=0.1)
    ix = _index(ghn, prob)
    q = _dev(prob.queries)
    with pytest.raises(ghn.GHNError) as e:
        ix.predict(q, 51)
    assert e.value.code == -3  # k > n
    empty = torch.empty((0, 2), dtype=torch.float32, device="cuda")
    out = ix.predict(empty, 3)
    assert out["idx"].shape == (0, 3)
    with pytest.raises(ghn.GHNError) as e:
        ix.predict(q, 65)
    assert e.value.code == -1
    with pytest.raises(ghn.GHNError) as e:
        ix.predict(q, 0)
    assert e.value.code == -1


# ---------------------------------------------------------------------------------- tree lookup
TREE = 1


@pytest.mark.parametrize("f", [1, 2, 3, 4, 5, 8])
def test_tree_lookup_uniform(ghn, f):
    width = {1: 0.003, 2: 0.05, 3: 0.1, 4: 0.2, 5: 0.3, 8: 0.5}[f]
    prob = W.uniform_problem(n=6000, m=301, f=f, k=9, seed=40 + f, width=width, q_lo=-0.3, q_hi=1.3)
    _check_exact(ghn, prob, lookup=TREE)
    _check_paper(ghn, prob, lookup=TREE)


def test_tree_lookup_edge_cases(ghn):
    lat = W.lattice_problem(n=3000, m=300, f=3, k=12, seed=7)
    _check_exact(ghn, lat, lookup=TREE)
    _check_paper(ghn, lat, lookup=TREE)
    far = W.uniform_problem(n=5000, m=120, f=3, k=5, seed=5, width=0.1)
    far.queries[:40] *= 1e3
    far.queries[40:80] -= 37.0
    _check_exact(ghn, far, lookup=TREE)
    _check_paper(ghn, far, lookup=TREE)
    one = W.uniform_problem(n=1, m=20, f=2, k=1, seed=3, width=0.5, q_lo=-5, q_hi=5)
    _check_exact(ghn, one, lookup=TREE)
    _check_paper(ghn, one, lookup=TREE)
    reg = W.uniform_problem(n=8000, m=200, f=3, k=16, seed=4, task=W.REGRESS, width=0.05)
    _check_exact(ghn, reg, lookup=TREE)
    widths = np.array([0.31, 0.07, 0.19], np.float32)
    origin = np.array([-0.123, 0.05, 1.7], np.float32)
    wo = W.uniform_problem(n=8000, m=200, f=3, k=9, seed=21, lo=-2.0, hi=2.0, q_lo=-3.0, q_hi=3.0)
    _check_exact(ghn, wo, widths=widths, origin=origin, lookup=TREE)
    _check_paper(ghn, wo, widths=widths, origin=origin, lookup=TREE)


def test_tree_equals_dense(ghn):
    prob = W.make("clusters4d", n=40_000, m=2_000)
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        a = _run(ghn, _index(ghn, prob, lookup=0), prob.queries, prob.k, stop)
        b = _run(ghn, _index(ghn, prob, lookup=TREE), prob.queries, prob.k, stop)
        _assert_same(a, b, "dense vs tree", check_layers=True)


def test_tree_walk_many_layers_and_pending_overflow(ghn):
    """Multi-layer tree walks against the grid oracle, stop layers included: the
    skewed 8-D mix (uniform-background queries walk up to about ten layers) and
    sparse 12-D data with k = 64, where a query defers more blocks to later layers
    than the per-wave pending list holds (those walks fall back to walking every
    later layer from the root).  The 12-D grid also fits the dense table, whose
    walk shares no lookup code with the tree."""
    skew = W.make("skew8d", n=200_000, m=400)
    assert _index(ghn, skew).info.lookup == TREE
    wide = W.uniform_problem(n=400_000, m=160, f=12, k=64, seed=77, width=0.3)
    for prob in (skew, wide):
        ix = _index(ghn, prob, lookup=TREE)
        g = oracle.Grid(prob.points_f32(), prob.targets, prob.task, prob.cell_width)
        for stop, ostop in ((ghn.GHN_STOP_EXACT, oracle.STOP_EXACT), (ghn.GHN_STOP_PAPER, oracle.STOP_PAPER)):
            got = _run(ghn, ix, prob.queries, prob.k, stop)
            want = g.predict(prob.queries, prob.k, ostop)
            _assert_same(got, want, "%s tree walk, stop %d" % (prob.name, stop), check_layers=True)
            if prob is wide:
                dense = _run(ghn, _index(ghn, prob, lookup=0), prob.queries, prob.k, stop)
                _assert_same(got, dense, "12-D tree vs dense, stop %d" % stop, check_layers=True)
        g.close()


# ---------------------------------------------------------------------------------- hash lookup
HASH = 2


@pytest.mark.parametrize("f", [1, 2, 3, 4, 5, 8])
def test_hash_lookup_uniform(ghn, f):
    width = {1: 0.003, 2: 0.05, 3: 0.1, 4: 0.2, 5: 0.3, 8: 0.5}[f]
    prob = W.uniform_problem(n=6000, m=301, f=f, k=9, seed=70 + f, width=width, q_lo=-0.3, q_hi=1.3)
    ix, _ = _check_exact(ghn, prob, lookup=HASH)
    assert ix.info.lookup == HASH
    _check_paper(ghn, prob, lookup=HASH)


def test_hash_lookup_edge_cases(ghn):
    lat = W.lattice_problem(n=3000, m=300, f=3, k=12, seed=17)
    _check_exact(ghn, lat, lookup=HASH)
    _check_paper(ghn, lat, lookup=HASH)
    far = W.uniform_problem(n=5000, m=120, f=3, k=5, seed=15, width=0.1)
    far.queries[:40] *= 1e3
    far.queries[40:80] -= 37.0
    _check_exact(ghn, far, lookup=HASH)
    _check_paper(ghn, far, lookup=HASH)
    one = W.uniform_problem(n=1, m=20, f=2, k=1, seed=13, width=0.5, q_lo=-5, q_hi=5)
    _check_exact(ghn, one, lookup=HASH)
    _check_paper(ghn, one, lookup=HASH)
    widths = np.array([0.31, 0.07, 0.19], np.float32)
    origin = np.array([-0.123, 0.05, 1.7], np.float32)
    wo = W.uniform_problem(n=8000, m=200, f=3, k=9, seed=121, lo=-2.0, hi=2.0, q_lo=-3.0, q_hi=3.0)
    _check_exact(ghn, wo, widths=widths, origin=origin, lookup=HASH)
    _check_paper(ghn, wo, widths=widths, origin=origin, lookup=HASH)


def test_hash_equals_dense_and_tree(ghn):
    """Same neighbours, stop layers and candidate counts as the dense table (the walk
    enumerates the same runs); the same results as the tree."""
    prob = W.make("clusters4d", n=40_000, m=2_000)
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        a = _run(ghn, _index(ghn, prob, lookup=0), prob.queries, prob.k, stop)
        b = _run(ghn, _index(ghn, prob, lookup=HASH), prob.queries, prob.k, stop)
        c = _run(ghn, _index(ghn, prob, lookup=TREE), prob.queries, prob.k, stop)
        _assert_same(b, a, "hash vs dense", check_layers=True)
        assert np.array_equal(a["cands"], b["cands"])
        _assert_same(b, c, "hash vs tree", check_layers=True)


def test_hash_fine_grid_against_oracle(ghn):
    """A grid too fine for the dense table (about 0.1 points per cell): several
    layers per query, every generated cell looked up."""
    prob = W.make("clusters4d", n=200_000, m=400)
    width = 0.012
    ix = _index(ghn, prob, widths=width, lookup=HASH)
    assert ix.info.lookup == HASH and ix.info.box_cells > 16 * prob.n
    g = oracle.Grid(prob.points, prob.targets, prob.task, width)
    for stop, ostop in ((ghn.GHN_STOP_EXACT, oracle.STOP_EXACT), (ghn.GHN_STOP_PAPER, oracle.STOP_PAPER)):
        got = _run(ghn, ix, prob.queries, prob.k, stop)
        _assert_same(got, g.predict(prob.queries, prob.k, ostop), "fine hash grid, stop %d" % stop, check_layers=True)
        assert got["stop_layer"].max() >= 2
    g.close()


def test_hash_index_in_batches_bf16_and_save_load(ghn):
    import torch
    prob = W.uniform_problem(n=20_000, m=500, f=3, k=7, seed=91, width=0.04)
    ix = _index(ghn, prob, lookup=HASH)
    want = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT)
    # grouped bf16 screen (walks the index's tree)
    _assert_same(_run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT, prec=MFMA), want, "hash index, bf16")
    # persistent launch (tree walk for hash items)
    oi = torch.full((prob.m, prob.k), -7, dtype=torch.int64, device="cuda")
    op = torch.full((prob.m,), -7, dtype=torch.int32, device="cuda")
    od = torch.zeros((prob.m, prob.k), dtype=torch.float64, device="cuda")
    q = _dev(prob.queries)
    items = [(ix.handle, q, prob.k, oi, op, od)]
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    _assert_same(dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy()), want, "hash index, batch")
    # save / load keeps the lookup
    ix2 = ghn.Index.load(ix.save())
    assert ix2.info.lookup == HASH
    _assert_same(_run(ghn, ix2, prob.queries, prob.k, ghn.GHN_STOP_EXACT), want, "hash index, reloaded")


def test_hash_key_overflow_refused(ghn):
    # cell ids up to 1e8 (inside the +-2^27 id range) in 3 dimensions: a box of about
    # 1e24 cells, beyond the 2^62 of the hash keys
    pts = np.random.default_rng(3).random((500, 3)).astype(np.float32)
    with pytest.raises(ghn.GHNError) as e:
        ghn.Index(_dev(pts), _dev(np.zeros(500, np.int32)), 0, 1e-8, lookup=HASH)
    assert e.value.code == -5 and "hash" in str(e.value)


def test_skew8d_regression_small(ghn):
    prob = W.make("skew8d", n=100_000, m=1_000)
    ix, _ = _check_exact(ghn, prob)
    assert ix.info.lookup == TREE
    _check_paper(ghn, prob, sample=300)


def test_bf16_16d_small(ghn):
    prob = W.make("bf16_16d", n=60_000, m=600)
    ix, _ = _check_exact(ghn, prob)
    assert ix.info.lookup == TREE
    _check_paper(ghn, prob, sample=200)


# ---------------------------------------------------------------------------------- bf16 MFMA form
MFMA = 1


def _check_mfma(ghn, prob, sample=None, levels=-1, lookup=None, paper=True, seed=0, group_size=0, tile_width=0):
    ix = _index(ghn, prob, lookup=lookup)
    got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT, prec=MFMA, group_levels=levels,
               group_size=group_size, tile_width=tile_width)
    rows = np.arange(prob.m)
    if sample is not None and sample < prob.m:
        rows = np.sort(np.random.default_rng(seed).choice(prob.m, sample, replace=False))
    bi, bd, bp = oracle.bruteforce(prob.points_f32(), prob.targets, prob.task, prob.queries[rows], prob.k)
    _assert_same({k: v[rows] for k, v in got.items()}, dict(idx=bi, d2=bd, pred=bp), prob.name + " MFMA EXACT")
    if paper:
        gp = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_PAPER, prec=MFMA, group_size=group_size,
                  tile_width=tile_width)
        want = oracle.Grid(prob.points_f32(), prob.targets, prob.task, prob.cell_width).predict(
            prob.queries[rows], prob.k, oracle.STOP_PAPER)
        _assert_same({k: v[rows] for k, v in gp.items()}, want, prob.name + " MFMA PAPER", check_layers=True)
    return ix, got


def test_mfma_blobs2d(ghn):
    _check_mfma(ghn, W.make("blobs2d"))


def test_mfma_clusters4d_small(ghn):
    prob = W.make("clusters4d", n=60_000, m=3_001)
    for levels in (-1, 0, 2):
        _check_mfma(ghn, prob, levels=levels, paper=levels == -1)


@pytest.mark.parametrize("group_size,tile_width", [(1, 0), (4, 0), (8, 0), (0, 32), (4, 32)])
def test_mfma_group_sizes(ghn, group_size, tile_width):
    """Groups of at most 1, 4 or 8 queries (the tile's other query rows stay empty), and
    tiles of 32 candidates (two column blocks) instead of 64."""
    prob = W.make("clusters4d", n=40_000, m=1_500)
    _check_mfma(ghn, prob, levels=2, group_size=group_size, tile_width=tile_width)
    probs = _multi(problems=6, n_hi=20_000, m_hi=1_500, seed=61)
    idxs = [_index(ghn, p) for p in probs]
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        got = _batch_run_gs(ghn, probs, idxs, stop, group_size, tile_width)
        for i, (p, g) in enumerate(zip(probs, got)):
            _assert_same(g, _oracle_want(p, stop), "bf16 batch group_size=%d tile_width=%d item %d" % (
                group_size, tile_width, i))


@pytest.mark.parametrize("k", [1, 17, 33, 64])
def test_mfma_tile_width_32_k_values(ghn, k):
    """32-candidate tiles over every buffer width (one, two and four registers per
    16-lane row), with ragged tails: n and m are not multiples of the tile."""
    prob = W.uniform_problem(n=4_999, m=301, f=3, k=k, seed=260 + k, width=0.08)
    _check_mfma(ghn, prob, tile_width=32)


def _batch_run_gs(ghn, probs, idxs, stop, group_size, tile_width=0):
    import torch
    items, outs = [], []
    for p, ix in zip(probs, idxs):
        oi = torch.full((p.m, p.k), -7, dtype=torch.int64, device="cuda")
        op = torch.full((p.m,), -7, dtype=torch.int32, device="cuda")
        od = torch.zeros((p.m, p.k), dtype=torch.float64, device="cuda")
        items.append((ix.handle, _dev(p.queries), p.k, oi, op, od))
        outs.append((oi, op, od))
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, stop, MFMA), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, stop=stop, prec=MFMA, group_size=group_size, tile_width=tile_width)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    return [dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy()) for oi, op, od in outs]


@pytest.mark.parametrize("k", [1, 5, 16, 17, 32, 33, 64])
def test_mfma_k_values(ghn, k):
    prob = W.uniform_problem(n=5000, m=300, f=3, k=k, seed=200 + k, width=0.08)
    _check_mfma(ghn, prob)


def test_mfma_ties_far_nonfinite(ghn):
    lat = W.lattice_problem(n=3000, m=300, f=3, k=12, seed=5)
    _check_mfma(ghn, lat)
    reg = W.lattice_problem(n=3000, m=300, f=2, k=20, seed=6, task=W.REGRESS)
    _check_mfma(ghn, reg)
    far = W.uniform_problem(n=5000, m=200, f=3, k=5, seed=7, width=0.1)
    far.queries[:50] *= 1e3
    far.queries[50:90] -= 37.0
    _check_mfma(ghn, far)
    bad = W.uniform_problem(n=1000, m=40, f=2, k=3, seed=8, width=0.1)
    bad.queries[3, 1] = np.nan
    ix = _index(ghn, bad)
    got = _run(ghn, ix, bad.queries, bad.k, ghn.GHN_STOP_EXACT, prec=MFMA)
    assert (got["idx"][3] == -1).all() and got["pred"][3] == -1
    ok = np.delete(np.arange(bad.m), 3)
    bi, bd, bp = oracle.bruteforce(bad.points, bad.targets, bad.task, bad.queries[ok], bad.k)
    assert np.array_equal(got["idx"][ok], bi) and np.array_equal(got["d2"][ok], bd)


@pytest.mark.parametrize("f", [1, 2, 4, 5, 8])
def test_mfma_dims(ghn, f):
    width = {1: 0.003, 2: 0.05, 4: 0.2, 5: 0.3, 8: 0.5}[f]
    prob = W.uniform_problem(n=6000, m=301, f=f, k=9, seed=300 + f, width=width, q_lo=-0.3, q_hi=1.3)
    _check_mfma(ghn, prob)


def test_mfma_skew8d_and_bf16_16d(ghn):
    _check_mfma(ghn, W.make("skew8d", n=100_000, m=1_000), sample=300)
    _check_mfma(ghn, W.make("bf16_16d", n=60_000, m=600), sample=200)


# ---------------------------------------------------------------------------------- batches
def _multi(problems=20, n_hi=30_000, m_hi=3_000, seed=5):
    return W.make_multi3d(problems=problems, n_hi=n_hi, m_hi=m_hi, seed=seed)


def _batch_setup(ghn, probs, stop):
    import torch
    idxs, items, outs = [], [], []
    for p in probs:
        ix = _index(ghn, p)
        q = _dev(p.queries)
        oi = torch.full((p.m, p.k), -7, dtype=torch.int64, device="cuda")
        op = torch.full((p.m,), -7, dtype=torch.int32 if p.task == W.CLASSIFY else torch.float32, device="cuda")
        od = torch.zeros((p.m, p.k), dtype=torch.float64, device="cuda")
        idxs.append(ix)
        items.append((ix.handle, q, p.k, oi, op, od))
        outs.append((oi, op, od))
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, stop=stop)
    return idxs, items, outs, ws, batch


def test_batched_matches_single_and_oracle(ghn):
    import torch
    probs = _multi()
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        idxs, items, outs, ws, batch = _batch_setup(ghn, probs, stop)
        ghn.ghn_predict_batched(batch)
        torch.cuda.synchronize()
        for p, ix, (oi, op, od) in zip(probs, idxs, outs):
            single = _run(ghn, ix, p.queries, p.k, stop)
            got = dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy())
            _assert_same(got, single, "batched vs single")
            _assert_same(got, _oracle_want(p, stop), "batched vs oracle stop=%d" % stop)
        ghn.ghn_batch_destroy(batch)


def test_batched_tree_f8(ghn):
    """8-D tree indexes through the persistent launch (its f = 8 instance keeps the
    tree walk's pending list): three skewed problems of different sizes, against
    the single-index kernel and the oracle."""
    import torch
    probs = [W.make("skew8d", n=n, m=m, seed=s) for n, m, s in ((60_000, 700, 31), (150_000, 300, 32), (20_000, 900, 33))]
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        idxs, items, outs, ws, batch = _batch_setup(ghn, probs, stop)
        assert all(ix.info.lookup == TREE for ix in idxs)
        ghn.ghn_predict_batched(batch)
        torch.cuda.synchronize()
        for p, ix, (oi, op, od) in zip(probs, idxs, outs):
            got = dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy())
            _assert_same(got, _run(ghn, ix, p.queries, p.k, stop), "batched f=8 vs single")
            if stop == ghn.GHN_STOP_EXACT:
                rows = np.arange(min(p.m, 300))
                bi, bd, bp = oracle.bruteforce(p.points, p.targets, p.task, p.queries[rows], p.k)
                _assert_same({k: v[rows] for k, v in got.items()}, dict(idx=bi, d2=bd, pred=bp),
                             "batched f=8 vs oracle")
        ghn.ghn_batch_destroy(batch)


def _oracle_want(p, stop, median=False):
    """The oracle's answer for problem p: brute force (EXACT) or the grid walk (PAPER)."""
    task = oracle.REGRESS_MEDIAN if median else p.task
    pf = p.points_f32()
    if stop == 0:
        bi, bd, bp = oracle.bruteforce(pf, p.targets, task, p.queries, p.k)
        return dict(idx=bi, d2=bd, pred=bp)
    w = oracle.Grid(pf, p.targets, task, p.cell_width).predict(p.queries, p.k, oracle.STOP_PAPER)
    return dict(idx=w["idx"], d2=w["d2"], pred=w["pred"])


def _batch_run(ghn, probs, idxs, stop, prec, levels=-1, flags=0):
    """One batch over (problem, index) pairs; returns the host outputs per problem."""
    import torch
    items, outs = [], []
    for p, ix in zip(probs, idxs):
        q = _dev(p.queries)
        oi = torch.full((p.m, p.k), -7, dtype=torch.int64, device="cuda")
        op = torch.full((p.m,), -7, dtype=torch.int32 if p.task == W.CLASSIFY else torch.float32, device="cuda")
        od = torch.zeros((p.m, p.k), dtype=torch.float64, device="cuda")
        items.append((ix.handle, q, p.k, oi, op, od))
        outs.append((oi, op, od))
    nb = ghn.ghn_batch_workspace_bytes_for(items, stop, prec, flags, levels)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, stop=stop, flags=flags, prec=prec, group_levels=levels)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    return [dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy()) for oi, op, od in outs]


def test_batched_bf16_matches_oracle(ghn):
    """The bf16 screen over all items in one grouped persistent launch: every query of
    every problem against the oracle, both rules, several group sizes."""
    probs = _multi()
    idxs = [_index(ghn, p) for p in probs]
    for stop, levels in ((ghn.GHN_STOP_EXACT, -1), (ghn.GHN_STOP_EXACT, 0), (ghn.GHN_STOP_EXACT, 3),
                         (ghn.GHN_STOP_PAPER, -1)):
        got = _batch_run(ghn, probs, idxs, stop, MFMA, levels)
        for i, (p, g) in enumerate(zip(probs, got)):
            _assert_same(g, _oracle_want(p, stop), "bf16 batch item %d stop=%d levels=%d" % (i, stop, levels))


def test_batched_bf16_mixed_lookups_large_k_and_empty_item(ghn):
    probs = [W.uniform_problem(n=n, m=m, f=3, k=k, seed=s, width=0.05) for n, m, k, s in
             ((20_000, 400, 5, 161), (8_000, 300, 40, 162), (30_000, 0, 3, 163), (12_000, 350, 64, 164),
              (5_000, 200, 1, 165))]
    lookups = [0, TREE, 0, HASH, 0]
    idxs = [_index(ghn, p, lookup=lk) for p, lk in zip(probs, lookups)]
    assert [ix.info.lookup for ix in idxs] == lookups
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        got = _batch_run(ghn, probs, idxs, stop, MFMA)
        for i, (p, g) in enumerate(zip(probs, got)):
            if p.m:
                _assert_same(g, _oracle_want(p, stop), "mixed bf16 batch item %d stop=%d" % (i, stop))


def test_batched_bf16_regression_median(ghn):
    probs = [W.uniform_problem(n=n, m=m, f=3, k=k, seed=s, width=0.05, task=W.REGRESS) for n, m, k, s in
             ((15_000, 300, 6, 171), (9_000, 250, 11, 172), (4_000, 100, 20, 173))]
    idxs = [_index(ghn, p) for p in probs]
    for median in (False, True):
        got = _batch_run(ghn, probs, idxs, ghn.GHN_STOP_EXACT, MFMA, flags=ghn.GHN_FLAG_MEDIAN if median else 0)
        for i, (p, g) in enumerate(zip(probs, got)):
            _assert_same(g, _oracle_want(p, 0, median), "bf16 batch regression item %d median=%d" % (i, median))


def test_batched_bf16_graph_replay(ghn):
    import torch
    probs = _multi(problems=12, n_hi=20_000, m_hi=2_000, seed=29)
    items, outs = [], []
    idxs = [_index(ghn, p) for p in probs]
    for p, ix in zip(probs, idxs):
        oi = torch.empty((p.m, p.k), dtype=torch.int64, device="cuda")
        op = torch.empty(p.m, dtype=torch.int32, device="cuda")
        od = torch.empty((p.m, p.k), dtype=torch.float64, device="cuda")
        items.append((ix.handle, _dev(p.queries), p.k, oi, op, od))
        outs.append((oi, op, od))
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, prec=MFMA), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, prec=MFMA)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    want = [(oi.clone(), op.clone(), od.clone()) for oi, op, od in outs]
    for p, (wi, wp, wd) in zip(probs, want):
        _assert_same(dict(idx=wi.cpu().numpy(), pred=wp.cpu().numpy(), d2=wd.cpu().numpy()), _oracle_want(p, 0),
                     "bf16 batch before capture")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ghn.ghn_predict_batched(batch)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for oi, op, od in outs:      # eager work between replays
            oi.fill_(-1); op.fill_(-1); od.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (oi, op, od), (wi, wp, wd) in zip(outs, want):
            assert torch.equal(oi, wi) and torch.equal(op, wp) and torch.equal(od, wd), rep
    ghn.ghn_batch_destroy(batch)


def test_batched_mixed_lookups(ghn):
    """A batch of 3-D indexes where one uses the cell tree and the others the dense
    table (the launch then takes the instance that walks both)."""
    import torch
    probs = [W.uniform_problem(n=n, m=m, f=3, k=k, seed=s, width=0.05) for n, m, k, s in
             ((20_000, 400, 5, 61), (8_000, 300, 12, 62), (30_000, 500, 1, 63))]
    idxs, items, outs = [], [], []
    for i, p in enumerate(probs):
        ix = _index(ghn, p, lookup=TREE if i == 1 else 0)
        oi = torch.full((p.m, p.k), -7, dtype=torch.int64, device="cuda")
        op = torch.full((p.m,), -7, dtype=torch.int32, device="cuda")
        od = torch.zeros((p.m, p.k), dtype=torch.float64, device="cuda")
        q = _dev(p.queries)
        idxs.append((ix, q))
        items.append((ix.handle, q, p.k, oi, op, od))
        outs.append((oi, op, od))
    assert [ix.info.lookup for ix, _ in idxs] == [0, TREE, 0]
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items), dtype=torch.uint8, device="cuda")
        batch = ghn.ghn_batch_prepare(items, ws, stop=stop)
        ghn.ghn_predict_batched(batch)
        torch.cuda.synchronize()
        ghn.ghn_batch_destroy(batch)
        for p, (ix, _), (oi, op, od) in zip(probs, idxs, outs):
            got = dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy())
            _assert_same(got, _run(ghn, ix, p.queries, p.k, stop), "mixed batch vs single")
            _assert_same(got, _oracle_want(p, stop), "mixed batch vs oracle")


def test_batched_graph_replay(ghn):
    import torch
    probs = _multi(problems=12, n_hi=20_000, m_hi=2_000, seed=9)
    idxs, items, outs, ws, batch = _batch_setup(ghn, probs, ghn.GHN_STOP_EXACT)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    want = [(oi.clone(), op.clone(), od.clone()) for oi, op, od in outs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ghn.ghn_predict_batched(batch)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for oi, op, od in outs:      # eager work between replays
            oi.fill_(-1); op.fill_(-1); od.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (oi, op, od), (wi, wp, wd) in zip(outs, want):
            assert torch.equal(oi, wi) and torch.equal(op, wp) and torch.equal(od, wd), rep
    ghn.ghn_batch_destroy(batch)


def test_many_indexes_bf16_in_one_graph(ghn):
    """The grouped bf16 predicts of many indexes captured in one graph: every replay
    (with eager work in between) equals the eager calls."""
    import torch
    probs = _multi(problems=10, n_hi=30_000, m_hi=3_000, seed=19)
    runs = []
    for p in probs:
        ix = _index(ghn, p)
        q = _dev(p.queries)
        oi = torch.empty((p.m, p.k), dtype=torch.int64, device="cuda")
        op = torch.empty(p.m, dtype=torch.int32, device="cuda")
        nb = ghn.ghn_predict_workspace_bytes(ix.handle, p.m, p.k, ghn.GHN_STOP_EXACT, MFMA, 0)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
        runs.append((p, ix, q, oi, op, ws))

    def all_predicts():
        for p, ix, q, oi, op, ws in runs:
            ghn.ghn_predict(ix.handle, q, p.k, oi, op, None, ghn.GHN_STOP_EXACT, MFMA, 0, ws=ws)

    all_predicts()
    torch.cuda.synchronize()
    want = [(oi.clone(), op.clone()) for _, _, _, oi, op, _ in runs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            all_predicts()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for _, _, _, oi, op, ws in runs:
            oi.fill_(-1); op.fill_(-1); ws.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, _, oi, op, _), (wi, wp) in zip(runs, want):
            assert torch.equal(oi, wi) and torch.equal(op, wp), rep
    for (p, _, _, _, _, _), (wi, wp) in zip(runs, want):
        rows = np.arange(min(p.m, 100))
        bi, bd, bp = oracle.bruteforce(p.points, p.targets, p.task, p.queries[rows], p.k)
        assert np.array_equal(wi.cpu().numpy()[rows], bi) and np.array_equal(wp.cpu().numpy()[rows], bp)


def test_batch_errors(ghn):
    import torch
    probs = _multi(problems=2, n_hi=5_000, m_hi=100, seed=1)
    idxs, items, outs, ws, batch = _batch_setup(ghn, probs, ghn.GHN_STOP_EXACT)
    ghn.ghn_batch_destroy(batch)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_batch_prepare(items, small)
    assert e.value.code == -6
    bad = list(items)
    h, q, k, oi, op, od = bad[0]
    bad[0] = (h, q, 10 ** 6, oi, op, od)
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_batch_prepare(bad, ws)
    assert e.value.code == -1
    p4 = W.uniform_problem(n=500, m=10, f=4, k=3, seed=2, width=0.2)
    ix4 = _index(ghn, p4)
    mixed = list(items) + [(ix4.handle, _dev(p4.queries), 3, oi, op, od)]
    ws2 = torch.empty(ghn.ghn_batch_workspace_bytes_for(mixed), dtype=torch.uint8, device="cuda")
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_batch_prepare(mixed, ws2)
    assert e.value.code == -1


# ---------------------------------------------------------------------------------- autotune
def test_autotune_exact_and_paper(ghn, tmp_path):
    import torch
    from paper_2004_02290_amd import autotune
    prob = W.make("clusters4d", n=50_000, m=2_000)
    pts, tgt, q = _dev(prob.points), _dev(prob.targets), _dev(prob.queries)
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(pts, tgt, prob.task, q, prob.k, ghn.GHN_STOP_EXACT, cache_path=cache)
    assert best["ms"] > 0 and best["cell_width"] > 0
    # widths x (8 FP32 settings: 2 walk orders x 4 ring schedules + bf16 at 4 grouping
    # levels x 3 group and tile shapes), plus the 8 FP32 settings on the hash lookup for
    # every width whose build chose the tree (4 dimensions)
    tree_widths = {t["cell_width"] for t in best["trials"] if t["lookup"] == TREE}
    assert len(best["trials"]) == 6 * 20 + 8 * len(tree_widths)
    assert {(t["group_size"], t["tile_width"]) for t in best["trials"] if t["prec"] == MFMA} == {
        (16, 64), (8, 64), (16, 32)}
    assert sum(t["lookup"] == HASH for t in best["trials"]) == 8 * len(tree_widths)
    assert {t["ring_step"] for t in best["trials"]} == {0, 1, 2}
    again = autotune.tune(pts, tgt, prob.task, q, prob.k, ghn.GHN_STOP_EXACT, cache_path=cache)
    assert again["cell_width"] == best["cell_width"]  # served from the cache
    # the tuned setting still returns the brute-force neighbours
    ix = ghn.Index(pts, tgt, prob.task, best["cell_width"], lookup=best["lookup"])
    got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT, prec=best["prec"], flags=best["flags"],
               group_levels=best["group_levels"], ring_step=best["ring_step"], group_size=best["group_size"],
               tile_width=best["tile_width"])
    bi, bd, bp = oracle.bruteforce(prob.points, prob.targets, prob.task, prob.queries, prob.k)
    _assert_same(got, dict(idx=bi, d2=bd, pred=bp), "autotuned EXACT")
    pb, trials = ghn.ghn_autotune(pts, tgt, prob.task, q, prob.k, ghn.GHN_STOP_PAPER, widths=[prob.cell_width])
    assert abs(pb["cell_width"] - prob.cell_width) < 1e-9 and len(trials) == 5
    with pytest.raises(ghn.GHNError) as e:
        ghn.ghn_autotune(pts, tgt, prob.task, q, prob.k, ghn.GHN_STOP_PAPER)
    assert e.value.code == -1


# ---------------------------------------------------------------------------------- far queries
def _far_problem(f, seed, n=3000, m=96, width=0.1, k=5):
    """Uniform points on [0, 1)^f (cell ids 0..9) and queries far outside in two or more
    dimensions at different distances: 2^29 .. 2^31 cells out (the walk then runs in a
    shifted frame), around 2^28 cells out (the frame's edge) and beyond 2^40 cells (ids
    saturate).  The first rows stay ordinary queries."""
    prob = W.uniform_problem(n=n, m=m, f=f, k=k, seed=seed, width=width)
    rng = np.random.default_rng(seed)
    q = prob.queries.astype(np.float64)
    cells = [2.0 ** 28 - 3, 2.0 ** 28, 2.0 ** 28 + 5, 2.0 ** 29, 3.1e8, 2.0 ** 30, 1.7e9, 2.0 ** 31, 2.0 ** 41,
             2.0 ** 45]
    for r in range(8, m):
        dims = rng.choice(f, size=min(f, int(rng.integers(2, f + 1))), replace=False)
        for j in dims:
            c = cells[int(rng.integers(0, len(cells)))] * (1.0 + 0.01 * rng.random())
            q[r, j] = (-c if rng.random() < 0.5 else c + 10.0) * width
    # two rows with every far dimension at the same distance
    q[8, :2] = -(2.0 ** 30) * width
    q[9, :] = (2.0 ** 29) * width
    prob.queries = q.astype(np.float32)
    return prob


@pytest.mark.parametrize("f", [2, 3, 4])
def test_far_queries_shifted_frame(ghn, f):
    prob = _far_problem(f, seed=40 + f)
    _check_exact(ghn, prob)
    got = _check_paper(ghn, prob)
    assert (got["stop_layer"][8:] > 2 ** 28).all()


@pytest.mark.parametrize("lookup", [TREE, HASH])
def test_far_queries_shifted_frame_other_lookups(ghn, lookup):
    prob = _far_problem(3, seed=50 + lookup)
    _check_exact(ghn, prob, lookup=lookup)
    _check_paper(ghn, prob, lookup=lookup)


def test_far_queries_shifted_frame_mfma(ghn):
    prob = _far_problem(3, seed=60)
    _check_mfma(ghn, prob)


def test_far_queries_shifted_frame_batched_bf16(ghn):
    probs = [_far_problem(3, seed=80 + i, n=1000 + 700 * i, m=40 + 9 * i) for i in range(4)]
    idxs = [_index(ghn, p) for p in probs]
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        for i, (p, g) in enumerate(zip(probs, _batch_run(ghn, probs, idxs, stop, MFMA))):
            _assert_same(g, _oracle_want(p, stop), "bf16 batch far queries item %d stop=%d" % (i, stop))


def test_far_queries_shifted_frame_batched(ghn):
    import torch
    probs = [_far_problem(3, seed=70 + i, n=1000 + 700 * i, m=40 + 9 * i) for i in range(4)]
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        idxs, items, outs, ws, batch = _batch_setup(ghn, probs, stop)
        ghn.ghn_predict_batched(batch)
        torch.cuda.synchronize()
        for p, ix, (oi, op, od) in zip(probs, idxs, outs):
            got = dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy())
            if stop == ghn.GHN_STOP_EXACT:
                bi, bd, bp = oracle.bruteforce(p.points, p.targets, p.task, p.queries, p.k)
                want = dict(idx=bi, d2=bd, pred=bp)
            else:
                w = oracle.Grid(p.points, p.targets, p.task, p.cell_width).predict(p.queries, p.k, oracle.STOP_PAPER)
                want = dict(idx=w["idx"], d2=w["d2"], pred=w["pred"])
            _assert_same(got, want, "batched far queries stop=%d" % stop)
        ghn.ghn_batch_destroy(batch)


def test_batched_independent_of_grid_and_order(ghn):
    """The persistent FP32 launch gives the same answers whatever its grid size (one
    block, a few, the default) and walk order (spatial or input order), for both rules;
    its answers are the oracle's."""
    import os
    probs = _multi(problems=16, n_hi=40_000, m_hi=3_000, seed=41)
    assert sum(p.m for p in probs) >= 4096  # large enough for the spatial order
    idxs = [_index(ghn, p) for p in probs]
    for stop in (ghn.GHN_STOP_EXACT, ghn.GHN_STOP_PAPER):
        want = [_oracle_want(p, stop) for p in probs]
        for blocks, flags in ((None, 0), ("1", 0), ("3", 0), ("5", ghn.GHN_FLAG_NO_SORT)):
            old = os.environ.pop("GHN_BATCH_BLOCKS", None)
            if blocks is not None:
                os.environ["GHN_BATCH_BLOCKS"] = blocks
            try:
                got = _batch_run(ghn, probs, idxs, stop, ghn.GHN_PREC_FP32, flags=flags)
            finally:
                os.environ.pop("GHN_BATCH_BLOCKS", None)
                if old is not None:
                    os.environ["GHN_BATCH_BLOCKS"] = old
            for i, (g, w) in enumerate(zip(got, want)):
                _assert_same(g, w, "batch item %d stop=%d blocks=%s flags=%d" % (i, stop, blocks, flags))


# ---------------------------------------------------------------------------------- ring schedule
@pytest.mark.parametrize("name,kw,lookup", [
    ("clusters4d", dict(n=60_000, m=1_500), None),                # dense table
    ("skew8d", dict(n=80_000, m=600, seed=5), None),              # cell tree
    ("clusters4d", dict(n=30_000, m=800), HASH),                  # hash lookup
    ("blobs2d", dict(), None),                                     # full size, the benchmark's ring 2
])
def test_ring_schedule_same_neighbours(ghn, name, kw, lookup):
    """EXACT walks that visit several layers per step (and double the step while the
    buffer is not full) return the brute-force neighbours; they stop no earlier than
    the layer-by-layer walk."""
    prob = W.make(name, **kw)
    ix = _index(ghn, prob, lookup=lookup)
    bi, bd, bp = oracle.bruteforce(prob.points_f32(), prob.targets, prob.task, prob.queries, prob.k)
    want = dict(idx=bi, d2=bd, pred=bp)
    base = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT)
    for step, flags in ((2, 0), (3, 0), (8, 0), (1, ghn.GHN_FLAG_RING_GROW), (2, ghn.GHN_FLAG_RING_GROW)):
        got = _run(ghn, ix, prob.queries, prob.k, ghn.GHN_STOP_EXACT, ring_step=step, flags=flags)
        _assert_same(got, want, "%s ring_step=%d flags=%d" % (name, step, flags))
        assert (got["stop_layer"] >= base["stop_layer"]).all()


def test_ring_schedule_batched_and_refused_under_paper(ghn):
    probs = _multi(problems=8, n_hi=30_000, m_hi=2_000, seed=51)
    idxs = [_index(ghn, p) for p in probs]
    for flags in (0, ghn.GHN_FLAG_NO_SORT):
        got = _batch_run_ring(ghn, probs, idxs, 4, ghn.GHN_FLAG_RING_GROW | flags)
        for i, (p, g) in enumerate(zip(probs, got)):
            _assert_same(g, _oracle_want(p, 0), "ring batch item %d" % i)
    p = probs[0]
    with pytest.raises(ghn.GHNError) as e:
        _run(ghn, idxs[0], p.queries, p.k, ghn.GHN_STOP_PAPER, ring_step=2)
    assert e.value.code == -1
    with pytest.raises(ghn.GHNError) as e:
        _run(ghn, idxs[0], p.queries, p.k, ghn.GHN_STOP_PAPER, flags=ghn.GHN_FLAG_RING_GROW)
    assert e.value.code == -1


def _batch_run_ring(ghn, probs, idxs, ring_step, flags):
    import torch
    items, outs = [], []
    for p, ix in zip(probs, idxs):
        oi = torch.full((p.m, p.k), -7, dtype=torch.int64, device="cuda")
        op = torch.full((p.m,), -7, dtype=torch.int32, device="cuda")
        od = torch.zeros((p.m, p.k), dtype=torch.float64, device="cuda")
        items.append((ix.handle, _dev(p.queries), p.k, oi, op, od))
        outs.append((oi, op, od))
    ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, flags=flags), dtype=torch.uint8, device="cuda")
    batch = ghn.ghn_batch_prepare(items, ws, flags=flags, ring_step=ring_step)
    ghn.ghn_predict_batched(batch)
    torch.cuda.synchronize()
    ghn.ghn_batch_destroy(batch)
    return [dict(idx=oi.cpu().numpy(), pred=op.cpu().numpy(), d2=od.cpu().numpy()) for oi, op, od in outs]
