"""The build's cells against the oracle (Eq. 1, Algorithm 1): every training point's
cell ids, the set of occupied cells and each cell's point count, read back from the
index with ghn_index_cells, must equal the oracle's exactly: the same cell for every
point (exact floor semantics included), each point in exactly one cell, and the same
num_cells."""
import numpy as np
import pytest

import oracle
from paper_2004_02290_amd import workloads as W

pytestmark = pytest.mark.gpu

TREE, HASH = 1, 2


@pytest.fixture(scope="module")
def ghn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_02290_amd import binding
    return binding


def _check_cells(ghn, points, widths, origin=None, lookup=None, bf16=False):
    import torch
    pts32 = np.ascontiguousarray(points, dtype=np.float32)
    if bf16:
        bits = (pts32.view(np.uint32) + 0x7FFF + ((pts32.view(np.uint32) >> 16) & 1)) >> 16  # round to nearest even
        pts32 = (bits.astype(np.uint32) << 16).view(np.float32)
        dev = torch.from_numpy(bits.astype(np.int16)).cuda().view(torch.bfloat16)
    else:
        dev = torch.from_numpy(pts32).cuda()
    n, f = pts32.shape
    tg = torch.zeros(n, dtype=torch.int32, device="cuda")
    ix = ghn.Index(dev, tg, ghn.GHN_CLASSIFY, widths, origin, lookup=lookup)
    ids, counts, point_cell = (t.cpu().numpy() for t in ghn.ghn_index_cells(ix.handle))
    g = oracle.Grid(pts32, np.zeros(n, np.int32), oracle.CLASSIFY, widths, origin)
    want_ids, want_counts = g.cells()
    assert ix.info.num_cells == g.num_cells == ids.shape[0]
    # the same occupied cells with the same counts (the index keeps its own cell order)
    order = np.lexsort(ids.T[::-1])
    assert np.array_equal(ids[order].astype(np.int64), want_ids)
    assert np.array_equal(counts[order], want_counts)
    assert counts.sum() == n and (counts > 0).all()
    # every point in its own cell (Eq. 1, exact floor)
    assert (point_cell >= 0).all() and (point_cell < ids.shape[0]).all()
    assert np.array_equal(ids[point_cell].astype(np.int64), oracle.cells(pts32, widths, origin))
    assert np.array_equal(np.bincount(point_cell, minlength=ids.shape[0]), counts)
    ix.close()


@pytest.mark.parametrize("lookup", [None, TREE, HASH])
def test_cells_clusters4d_full_size(ghn, lookup):
    prob = W.make("clusters4d")
    _check_cells(ghn, prob.points, prob.cell_width, lookup=lookup)


def test_cells_blobs2d_and_skew8d(ghn):
    prob = W.make("blobs2d")
    _check_cells(ghn, prob.points, prob.cell_width)
    prob = W.make("skew8d", n=300_000, m=10)
    _check_cells(ghn, prob.points, prob.cell_width)


def test_cells_bf16_points(ghn):
    prob = W.make("bf16_16d", n=200_000, m=10)
    _check_cells(ghn, prob.points_f32(), prob.cell_width, bf16=True)


def test_cells_adversarial_floors(ghn):
    """Coordinates where the rounded quotient is on the wrong side of an integer
    (1 // 0.1 = 9 although fl(1 / 0.1) = 10), exact multiples of the width and their
    float neighbours, negative zero, tiny values and negative coordinates."""
    rng = np.random.default_rng(21)
    base = np.array([1.0, -1.0, 0.3, 0.7, 3.0, -3.0, 0.0, -0.0, 1e-30, -1e-30, 2.5, 1e3, -1e3, 0.1, 0.2],
                    dtype=np.float32)
    for a in (0.1, 0.3, 0.7, 0.021281155, 1.0 / 3.0, 2.5e-3):
        af = np.float32(a)
        t = rng.integers(-2000, 2000, 3000)
        mult = (t * np.float64(af)).astype(np.float32)
        x = np.concatenate([base, mult, np.nextafter(mult, np.float32(np.inf)),
                            np.nextafter(mult, np.float32(-np.inf))])
        pts = np.stack([x, rng.permutation(x)], axis=1)
        for lookup in (None, TREE):
            _check_cells(ghn, pts, float(af), lookup=lookup)


def test_cells_per_dim_widths_and_origin(ghn):
    rng = np.random.default_rng(22)
    pts = rng.normal(0, 2, (50_000, 3)).astype(np.float32)
    widths = [0.05, 0.21, 0.013]
    origin = [-1.3, 0.7, 2.25]
    for lookup in (None, TREE, HASH):
        _check_cells(ghn, pts, widths, origin, lookup=lookup)
