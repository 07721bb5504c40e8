#!/usr/bin/env python3
"""Throughput of GHN predict on one MI355X.

A step is one ghn_predict call over the whole query batch: hash every query to
its central cell, walk the layers, screen, select the k nearest and vote (the
whole hot path).  The index is built and every input is resident in HBM
before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload clusters4d]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/sec at k=10 on 1 MI355X, BF16-batched vs FP32 form; % HBM/MFMA peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
PREDICT_SRC = os.path.join(ROOT, "paper_2004_02290_amd", "csrc", "ghn_predict.hip")


def describe(prob, stop_name):
    return ("%s: n=%d f=%d %s points, m=%d queries, k=%d, %s, %s stop, FP32 screen + FP64 boundary" % (
        prob.name, prob.n, prob.f, prob.dtype.upper(), prob.m, prob.k,
        "majority vote" if prob.task == 0 else "mean", stop_name))


def source_hash() -> str:
    with open(PREDICT_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if the kernel is unchanged."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get(workload)
    if not entry or entry.get("predict_source_sha256_16") != source_hash():
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline(prob, target_s: float = 15.0):
    """The oracle's grid walk (EXACT rule) on a bounded query sample, all host threads."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g = oracle.Grid(prob.points_f32(), prob.targets, prob.task, prob.cell_width)
    pilot = min(prob.m, max(64, 8 * threads))
    t0 = time.perf_counter()
    g.predict(prob.queries[:pilot], prob.k, oracle.STOP_EXACT, nthreads=threads)
    dt = time.perf_counter() - t0
    sample = int(min(prob.m, max(pilot, pilot * target_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    g.predict(prob.queries[:sample], prob.k, oracle.STOP_EXACT, nthreads=threads)
    dt = time.perf_counter() - t0
    g.close()
    return {"value": sample / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d queries, grid walk with EXACT stop (same method, FP64, OpenMP over queries)"
                      % (sample, prob.m)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clusters4d")
    ap.add_argument("--stop", default="exact", choices=["exact", "paper"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sort", action="store_true", help="walk queries in input order")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "launches": 3}))
        return

    from paper_2004_02290_amd import binding as ghn
    from paper_2004_02290_amd import workloads as W

    prob = W.make(args.workload)
    stop = ghn.GHN_STOP_EXACT if args.stop == "exact" else ghn.GHN_STOP_PAPER
    dev = torch.device("cuda:0")
    if prob.dtype == "bf16":
        pts = torch.from_numpy(prob.points.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        pts = torch.from_numpy(prob.points).to(dev)
    tgt = torch.from_numpy(prob.targets).to(dev)
    qs = torch.from_numpy(prob.queries).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    ix = ghn.Index(pts, tgt, prob.task, prob.cell_width)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3

    m, k = prob.m, prob.k
    out_idx = torch.empty((m, k), dtype=torch.int64, device=dev)
    out_pred = torch.empty(m, dtype=torch.int32 if prob.task == 0 else torch.float32, device=dev)

    # Work counts for the algorithmic byte figure (untimed pass with statistics).
    flags = ghn.GHN_FLAG_NO_SORT if args.no_sort else 0
    nws = ghn.ghn_predict_workspace_bytes(ix.handle, m, k, stop, ghn.GHN_PREC_FP32, flags)
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
    st = ix.predict(qs, k, stop=stop, flags=flags, with_d2=False, with_stats=True)
    torch.cuda.synchronize()
    cands = int(st["cands"].sum().item())
    probes = int(st["probes"].sum().item())
    layers = st["stop_layer"].double()
    del st

    # A step = spatial order of the batch (Morton sort) + the walk kernel.  Events
    # between the two calls time the walk kernel alone, on the stream both run on.
    order = torch.empty(m, dtype=torch.int32, device=dev)
    ows = torch.empty(max(ghn.ghn_query_order_workspace_bytes(m), 1), dtype=torch.uint8, device=dev)

    def step(ev_mid=None):
        if args.no_sort:
            if ev_mid is not None:
                ev_mid.record()
            ghn.ghn_predict(ix.handle, qs, k, out_idx, out_pred, None, stop, ghn.GHN_PREC_FP32, flags, ws=ws)
        else:
            ghn.ghn_query_order(ix.handle, qs, order, ows)
            if ev_mid is not None:
                ev_mid.record()
            ghn.ghn_predict(ix.handle, qs, k, out_idx, out_pred, None, stop, ghn.GHN_PREC_FP32, flags, order=order)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    evm = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for i in range(args.steps):
        ev0[i].record()
        step(evm[i])
        ev1[i].record()
    torch.cuda.synchronize()
    per = np.array([ev0[i].elapsed_time(ev1[i]) for i in range(args.steps)])
    walk = np.array([evm[i].elapsed_time(ev1[i]) for i in range(args.steps)])
    ms = float(ev0[0].elapsed_time(ev1[-1])) / args.steps
    walk_ms = float(walk.mean())

    f = prob.f
    alg_bytes = (m * 4 * f + cands * (4 * f + 4) + probes * 4 + m * k * 4 + m * k * 8 + m * 4)
    achieved = alg_bytes / (walk_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    line = {
        "metric": METRIC,
        "value": m / (ms * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(prob, args.stop.upper()), "n": prob.n, "f": f, "m": m, "k": k,
                   "cell_width": prob.cell_width, "stop": args.stop, "form": "fp32_plain",
                   "query_order": "input" if args.no_sort else "morton"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "forms": {"fp32_plain_qps": m / (ms * 1e-3), "bf16_batched_qps": None},
        "walk_kernel_ms": walk_ms,
        "step_ms_p10_p50_p90": [float(np.percentile(per, 10)), float(np.median(per)), float(np.percentile(per, 90))],
        "work": {"candidates_per_query": cands / m, "table_reads_per_query": probes / m,
                 "mean_stop_layer": float(layers.mean().item()), "algorithmic_bytes_per_step": alg_bytes},
        "build_ms": build_ms,
        "index": {"num_cells": int(ix.info.num_cells), "box_cells": int(ix.info.box_cells),
                  "max_occupancy": int(ix.info.max_occupancy)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
    ix.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
