"""Writes fullsize.npz: the oracle's answers for sampled rows of every workload at its
full size, stored as one 64-bit hash per row, for the GPU full-size parity tests.

Run from the repository root:  python tests/golden/make_fullsize.py
It calls only the oracle (brute force for the EXACT rule, the grid walk for the
PAPER rule, at each workload's calibrated cell width) and the seeded workload
generators.  Row sets (seeded):
  clusters4d  10,000 queries
  skew8d      2,000 queries of each half (cluster / uniform background)
  bf16_16d    2,000 queries
  multi3d     every query of 32 problems (seeded choice among those with m n <= 4e9)
A row's hash covers its neighbour ids (int64), FP64 distances and prediction, and
for the PAPER rule its stop layer (int32); see row_hashes.  A multi3d problem's rows
are folded into one hash per problem and rule (fold)."""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_02290_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "fullsize.npz")
MULTI_PROBLEMS = 32


def row_hashes(idx, d2, pred, stop_layer=None) -> np.ndarray:
    """One 64-bit BLAKE2b hash per row of (idx int64, d2 float64, pred, stop_layer int32)."""
    idx = np.ascontiguousarray(idx, dtype="<i8")
    d2 = np.ascontiguousarray(d2, dtype="<f8")
    pred = np.ascontiguousarray(pred)
    out = np.empty(idx.shape[0], dtype=np.uint64)
    for r in range(idx.shape[0]):
        h = hashlib.blake2b(digest_size=8)
        h.update(idx[r].tobytes())
        h.update(d2[r].tobytes())
        h.update(pred[r:r + 1].tobytes())
        if stop_layer is not None:
            h.update(np.asarray(stop_layer[r], dtype="<i4").tobytes())
        out[r] = np.frombuffer(h.digest(), dtype="<u8")[0]
    return out


def fold(hashes) -> np.uint64:
    """One 64-bit hash of a whole set of row hashes (a problem's every row, in order)."""
    h = hashlib.blake2b(np.ascontiguousarray(hashes, dtype="<u8").tobytes(), digest_size=8)
    return np.frombuffer(h.digest(), dtype="<u8")[0]


def sample_rows(prob, name):
    if name == "clusters4d":
        return np.sort(np.random.default_rng(31).choice(prob.m, 10_000, replace=False))
    if name == "skew8d":
        rng = np.random.default_rng(32)
        parts = [np.flatnonzero(prob.query_part == v) for v in (1, 0)]
        return np.sort(np.concatenate([rng.choice(p, 2_000, replace=False) for p in parts]))
    if name == "bf16_16d":
        return np.sort(np.random.default_rng(33).choice(prob.m, 2_000, replace=False))
    raise ValueError(name)


def multi_problems(probs):
    ok = [i for i, p in enumerate(probs) if p.m * p.n <= 4e9]
    return sorted(np.random.default_rng(34).choice(ok, MULTI_PROBLEMS, replace=False).tolist())


def answers(prob, rows):
    """(EXACT hashes, PAPER hashes) of the given query rows."""
    pts = prob.points_f32()
    q = prob.queries[rows]
    bi, bd, bp = oracle.bruteforce(pts, prob.targets, prob.task, q, prob.k)
    g = oracle.Grid(pts, prob.targets, prob.task, prob.cell_width)
    w = g.predict(q, prob.k, oracle.STOP_PAPER)
    g.close()
    return row_hashes(bi, bd, bp), row_hashes(w["idx"], w["d2"], w["pred"], w["stop_layer"])


def main():
    out = {}
    for name in ("clusters4d", "skew8d", "bf16_16d"):
        t0 = time.time()
        prob = W.make(name)
        rows = sample_rows(prob, name)
        ex, pa = answers(prob, rows)
        out[name + "/rows"] = rows.astype(np.int32)
        out[name + "/exact"] = ex
        out[name + "/paper"] = pa
        out[name + "/width"] = np.float32(prob.cell_width)
        print("%s: %d rows in %.0f s" % (name, rows.size, time.time() - t0), flush=True)
    t0 = time.time()
    probs = W.make_multi3d()
    chosen = multi_problems(probs)
    out["multi3d/problems"] = np.asarray(chosen, dtype=np.int32)
    ex_all, pa_all = [], []
    for i in chosen:
        p = probs[i]
        ex, pa = answers(p, np.arange(p.m))
        ex_all.append(fold(ex))
        pa_all.append(fold(pa))
    out["multi3d/exact"] = np.asarray(ex_all, dtype=np.uint64)
    out["multi3d/paper"] = np.asarray(pa_all, dtype=np.uint64)
    print("multi3d: %d problems, %d queries in %.0f s" % (len(chosen), sum(probs[i].m for i in chosen),
                                                          time.time() - t0), flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
