"""ghn_predict_noalloc, the entry point for callers that cannot allocate device
memory, against ghn_predict (caller workspace) on the same index and queries:
two calls in a row, the second with fewer queries, must give bit-identical
neighbours, distances, predictions and stop layers."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ghn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_02290_amd import binding
    return binding


def _outs(ghn, m, k, task):
    import torch
    return dict(idx=torch.full((m, k), -7, dtype=torch.int64, device="cuda"),
                pred=torch.full((m,), -7, dtype=torch.int32 if task == ghn.GHN_CLASSIFY else torch.float32,
                                device="cuda"),
                d2=torch.zeros((m, k), dtype=torch.float64, device="cuda"),
                stop_layer=torch.full((m,), -7, dtype=torch.int32, device="cuda"))


def _host(d):
    return {key: v.cpu().numpy() for key, v in d.items()}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("stop", [0, 1])
def test_noalloc_matches_predict_two_calls(ghn, prec, stop):
    import torch
    from paper_2004_02290_amd import workloads as W
    prob = W.make("clusters4d", n=200_000, m=20_000)
    ix = ghn.Index(torch.from_numpy(prob.points).cuda(), torch.from_numpy(prob.targets).cuda(), prob.task,
                   prob.cell_width)
    q = torch.from_numpy(prob.queries).cuda()
    sizes = (20_000, 5_000)  # the second call is smaller (both sort or group their queries)
    want = []
    for m in sizes:
        r = ix.predict(q[:m], prob.k, stop=stop, prec=prec, with_stats=True)
        want.append(_host({key: r[key] for key in ("idx", "pred", "d2", "stop_layer")}))
    got = []
    for m in sizes:
        o = _outs(ghn, m, prob.k, prob.task)
        ghn.ghn_predict_noalloc(ix.handle, q[:m], prob.k, o["idx"], o["pred"], o["d2"], stop=stop, prec=prec,
                                out_stop_layer=o["stop_layer"])
        got.append(o)
    torch.cuda.synchronize()
    for m, g, w in zip(sizes, got, want):
        g = _host(g)
        for key in ("idx", "pred", "d2", "stop_layer"):
            assert np.array_equal(g[key], w[key]), "m=%d %s differs (prec=%d stop=%d)" % (m, key, prec, stop)
    ix.close()


def test_noalloc_without_workspace_and_refusal(ghn):
    import torch
    from paper_2004_02290_amd import workloads as W
    prob = W.make("blobs2d", m=1000)
    ix = ghn.Index(torch.from_numpy(prob.points).cuda(), torch.from_numpy(prob.targets).cuda(), prob.task,
                   prob.cell_width)
    q = torch.from_numpy(prob.queries).cuda()
    # FP32 screen below the spatial-sort threshold: no workspace at all
    assert ghn.ghn_predict_workspace_bytes(ix.handle, 1000, prob.k) == 0
    r = ix.predict(q, prob.k)
    o = _outs(ghn, 1000, prob.k, prob.task)
    ghn.ghn_predict_noalloc(ix.handle, q, prob.k, o["idx"], o["pred"], o["d2"])
    torch.cuda.synchronize()
    for key in ("idx", "pred", "d2"):
        assert np.array_equal(o[key].cpu().numpy(), r[key].cpu().numpy()), key
    # more queries than the library's array can serve: refused on the host, nothing launched
    big = torch.zeros((2_000_000, 2), dtype=torch.float32, device="cuda")
    assert ghn.ghn_predict_workspace_bytes(ix.handle, big.shape[0], prob.k, prec=ghn.GHN_PREC_BF16_MFMA) > \
        ghn.GHN_NOALLOC_WS_BYTES
    ob = _outs(ghn, big.shape[0], prob.k, prob.task)  # full size, although nothing may be written
    with pytest.raises(ghn.GHNError) as err:
        ghn.ghn_predict_noalloc(ix.handle, big, prob.k, ob["idx"], ob["pred"], prec=ghn.GHN_PREC_BF16_MFMA)
    assert err.value.code == -6
    ix.close()
