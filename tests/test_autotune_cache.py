"""Host logic of the autotuning cache (no GPU: the timing call is replaced).

Under the PAPER rule the cell width decides which neighbours come back, so a
cached choice may only be reused for the width it was tuned at; the key also
separates data sets that share n, f and coordinate range.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2004_02290_amd import autotune  # noqa: E402
from paper_2004_02290_amd import binding as ghn  # noqa: E402


@pytest.fixture
def fake_tuner(monkeypatch):
    calls = []

    def fake(points, targets, task, queries, k, stop, widths=None):
        w = float(np.atleast_1d(widths)[0]) if widths is not None else 0.05 * (len(calls) + 1)
        calls.append((stop, None if widths is None else list(np.atleast_1d(widths))))
        best = dict(cell_width=w, lookup=0, prec=0, group_levels=-1, flags=0, ms=1.0)
        return best, [best]

    monkeypatch.setattr(ghn, "ghn_autotune", fake)
    return calls


def _data(seed, n=2000, f=3):
    rng = np.random.default_rng(seed)
    pts = torch.from_numpy(rng.random((n, f), dtype=np.float32))
    pts[0] = 0.0
    pts[1] = 1.0  # same coordinate range for every seed
    return pts, torch.zeros(n, dtype=torch.int32), pts[:64].clone()


def test_paper_width_is_part_of_the_key(fake_tuner, tmp_path):
    cache = str(tmp_path / "tune.json")
    pts, tgt, q = _data(1)
    a = autotune.tune(pts, tgt, 0, q, 5, ghn.GHN_STOP_PAPER, widths=[0.1], cache_path=cache)
    b = autotune.tune(pts, tgt, 0, q, 5, ghn.GHN_STOP_PAPER, widths=[0.2], cache_path=cache)
    assert np.float32(a["cell_width"]) == np.float32(0.1)
    assert np.float32(b["cell_width"]) == np.float32(0.2)
    assert len(fake_tuner) == 2  # the second width was tuned, not served from the cache
    c = autotune.tune(pts, tgt, 0, q, 5, ghn.GHN_STOP_PAPER, widths=[0.1], cache_path=cache)
    assert np.float32(c["cell_width"]) == np.float32(0.1) and len(fake_tuner) == 2  # cached


def test_exact_cache_separates_data_task_and_k(fake_tuner, tmp_path):
    cache = str(tmp_path / "tune.json")
    p1, t1, q1 = _data(2)
    p2, t2, q2 = _data(3)
    autotune.tune(p1, t1, 0, q1, 5, ghn.GHN_STOP_EXACT, cache_path=cache)
    autotune.tune(p1, t1, 0, q1, 5, ghn.GHN_STOP_EXACT, cache_path=cache)
    assert len(fake_tuner) == 1
    autotune.tune(p2, t2, 0, q2, 5, ghn.GHN_STOP_EXACT, cache_path=cache)  # same n, f, range
    autotune.tune(p1, t1.float(), 1, q1, 5, ghn.GHN_STOP_EXACT, cache_path=cache)
    autotune.tune(p1, t1, 0, q1, 7, ghn.GHN_STOP_EXACT, cache_path=cache)
    autotune.tune(p1, t1, 0, q1, 5, ghn.GHN_STOP_EXACT, widths=[0.3, 0.4], cache_path=cache)
    assert len(fake_tuner) == 5
