"""The walk fault word (ghn_walk_faults): every walk ends with k rows of the index, so
after any number of ordinary calls (every lookup, both screens and stop rules, the
batched launch, brute force) the word reads 0 and no row carries the short-walk stop
layer (-2).  The condition itself is never provoked on a GPU; the guard's logic is
tested on the CPU (tests/test_guard_cpu.py)."""
import numpy as np
import pytest

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


def test_fault_word_stays_clear(ghn):
    import torch
    # whatever ran before in this process must not have raised it either
    assert ghn.ghn_walk_faults() == 0
    assert ghn.ghn_walk_faults(clear=True) == 0
    prob = W.make("clusters4d", n=60_000, m=5_000)
    pts = torch.from_numpy(prob.points).cuda()
    tg = torch.from_numpy(prob.targets).cuda()
    q = torch.from_numpy(prob.queries).cuda()
    # a far query and one with a NaN coordinate (stop layer -1, never -2)
    q[0] = 1e6
    q[1, 2] = float("nan")
    for lookup in (None, 1, 2):
        ix = ghn.Index(pts, tg, prob.task, prob.cell_width, lookup=lookup)
        for stop in (EXACT, PAPER):
            for prec in (FP32, BF16):
                out = ix.predict(q, 16, stop=stop, prec=prec, with_stats=True)
                sl = out["stop_layer"].cpu().numpy()
                assert (sl != -2).all() and sl[1] == -1 and (np.delete(sl, 1) >= 0).all()
        out = ix.bruteforce(q[:500], 8)
        assert (out["idx"][2:].cpu().numpy() >= 0).all()
        m = 3000
        oi = torch.empty((m, 12), dtype=torch.int64, device="cuda")
        op = torch.empty(m, dtype=torch.int32, device="cuda")
        od = torch.empty((m, 12), dtype=torch.float64, device="cuda")
        items = [(ix.handle, q[2:2 + m], 12, oi, op, od)]
        for stop in (EXACT, PAPER):
            for prec in (FP32, BF16):
                ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, stop, prec, 0), dtype=torch.uint8,
                                 device="cuda")
                batch = ghn.ghn_batch_prepare(items, ws, stop, prec=prec)
                ghn.ghn_predict_batched(batch)
                torch.cuda.synchronize()
                ghn.ghn_batch_destroy(batch)
                assert (oi.cpu().numpy() >= 0).all()
        ix.close()
    torch.cuda.synchronize()
    assert ghn.ghn_walk_faults() == 0
