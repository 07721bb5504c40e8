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
MFMA_BF16_PEAK_TFLOPS = 2500.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# workloads whose cell width the benchmark tunes before timing (the results do not depend on it
# under the EXACT rule): the skewed 8-D mix asks for it, and the 16-D bf16 clusters have no
# prescribed width
AUTOTUNED = ("skew8d", "bf16_16d")
CSRC = os.path.join(ROOT, "paper_2004_02290_amd", "csrc")


def describe(prob, stop_name):
    return ("%s: n=%d f=%d %s points, m=%d queries, k=%d, %s, %s stop" % (
        prob.name, prob.n, prob.f, prob.dtype.upper(), prob.m, prob.k,
        "majority vote" if prob.task == 0 else "mean", stop_name))


# Sources each walk kernel is compiled from (its traffic figure is void once they change).
KERNEL_SOURCES = {
    "k_predict_dense": ["ghn_predict.hip", "ghn_walk_dense.h", "ghn_walk.h", "ghn_guard.h", "ghn_internal.h"],
    "k_predict_tree": ["ghn_tree.hip", "ghn_walk_tree.h", "ghn_walk.h", "ghn_guard.h", "ghn_internal.h"],
    "k_predict_group": ["ghn_group.hip", "ghn_walk.h", "ghn_guard.h", "ghn_internal.h"],
    "k_predict_batched": ["ghn_batch.hip", "ghn_walk_dense.h", "ghn_walk_tree.h", "ghn_walk.h", "ghn_guard.h",
                          "ghn_internal.h"],
}


def source_hash(kernel: str) -> str:
    """Hash of the HIP sources of `kernel` (the code the counters were taken on)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, form: str, run=None, calibrated_width=None):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if the kernel is unchanged
    and the counters were taken in this run's configuration.

    `run` holds this run's settings (cell_width, and ring_step, ring_grow, sort for the FP32 walk
    or group_levels for the bf16 screen); an entry's recorded `config` must agree with every
    setting it records (a recorded cell width of None stands for `calibrated_width`)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get("%s/%s" % (workload, form))
    if not entry or entry.get("kernel") not in KERNEL_SOURCES:
        return None
    if entry.get("source_sha256_16") != source_hash(entry["kernel"]):
        return None
    cfg = entry.get("config")
    if cfg is not None and run is not None:
        for key, want in cfg.items():
            if key not in run:
                continue
            if key == "cell_width":
                w = calibrated_width if want is None else want
                if w is None or abs(float(run[key]) - float(w)) > 1e-6 * abs(float(w)):
                    return None
            elif run[key] != want:
                return None
    return entry.get("bytes_per_launch")


def traffic_config(args, form: str) -> dict:
    """Settings of a profiler run of `form` (bench.py arguments), recorded with its counters."""
    cfg = {"cell_width": args.cell_width}
    if form.startswith("fp32"):
        cfg.update(ring_step=args.ring_step if args.ring_step >= 0 else 2, ring_grow=bool(args.ring_grow),
                   sort=bool(args.sort))
    else:
        cfg.update(group_levels=args.group_levels, group_size=args.group_size or 16, tile_width=args.tile_width or 64)
    return cfg


# Algorithmic bytes of the gather/probe walk per query: 4f per candidate point gathered, 16 per
# index entry read, 4f for the query and 12k for the outputs (ids and distances); C_q and P_q
# are the kernels' own counts.  The extended count adds the 4-byte row id of every candidate
# and the prediction.
BYTES_FORMULA = "4f C_q + 16 P_q + 4f + 12k per query (C_q candidates, P_q index entries read)"


def walk_bytes(m, f, k, cands, probes):
    return m * 4 * f + cands * 4 * f + probes * 16 + m * 12 * k


def walk_bytes_extended(m, f, k, cands, probes):
    return m * 4 * f + cands * (4 * f + 4) + probes * 4 + m * k * 4 + m * k * 8 + m * 4


def hbm_roofline(alg_bytes, ext_bytes, kern_ms, traffic, kernel):
    """Roofline of a gather/probe kernel: `achieved` = algorithmic bytes / kernel time; the
    counter-measured HBM rate (FETCH_SIZE + WRITE_SIZE, which count L2 misses including those
    the Infinity Cache serves) and the extended byte count are reported beside it."""
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
         "traffic": traffic, "kernel": kernel, "bytes_per_launch": alg_bytes, "bytes_formula": BYTES_FORMULA,
         "achieved_extended": ext_bytes / (kern_ms * 1e-3) / 1e9}
    if traffic is not None:
        r["measured_GBs"] = traffic / (kern_ms * 1e-3) / 1e9
        r["traffic_over_algorithmic"] = traffic / alg_bytes
    return r


def write_traffic(pmc_dir: str, workloads, out_file: str = TRAFFIC_FILE, args=None) -> dict:
    """Turn rocprofv3 --pmc runs into HBM bytes per launch (profiles/traffic.json).

    Expects <pmc_dir>/<tag>/pmc_counter_collection.csv for the tags fetch_copy,
    write_copy (FETCH_SIZE / WRITE_SIZE of `bench.py --copy-calib`) and
    fetch_<workload>, write_<workload> (the same counters over a bench run).  The
    counters (KiB per dispatch) are scaled by what they read for the 1 GiB copy.
    Entries of other workloads already in the file are kept.
    """
    import csv

    def values(tag, name_part):
        with open(os.path.join(pmc_dir, tag, "pmc_counter_collection.csv")) as fh:
            return [float(r["Counter_Value"]) for r in csv.DictReader(fh) if name_part in r["Kernel_Name"]]

    copy_bytes = float(1 << 30)
    cf, cw = values("fetch_copy", "copyBuffer"), values("write_copy", "copyBuffer")
    fetch_scale = copy_bytes / (float(np.mean(cf)) * 1024.0)
    write_scale = copy_bytes / (float(np.mean(cw)) * 1024.0)
    try:
        with open(out_file) as fh:
            out = json.load(fh)
    except (OSError, ValueError):
        out = {}
    out["copy_calibration"] = {"bytes": copy_bytes, "fetch_kib": float(np.mean(cf)), "write_kib": float(np.mean(cw)),
                               "fetch_scale": fetch_scale, "write_scale": write_scale}
    for w in workloads:
        for form, kname in (("fp32", "k_predict_dense"), ("fp32", "k_predict_tree"), ("bf16", "k_predict_group"),
                            ("fp32_batched", "k_predict_batched")):
            fv, wv = values("fetch_" + w, kname), values("write_" + w, kname)
            if not fv or not wv:
                continue
            fk, wk = float(np.mean(fv)), float(np.mean(wv))
            out["%s/%s" % (w, form)] = {
                "kernel": kname, "dispatches": len(fv), "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
                "bytes_per_launch": fk * 1024.0 * fetch_scale + wk * 1024.0 * write_scale,
                "source_sha256_16": source_hash(kname)}
            if args is not None and w != "multi3d":
                out["%s/%s" % (w, form)]["config"] = traffic_config(args, form)
    with open(out_file, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))
    return out


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


def paper_study(args, ghn, W, torch):
    """The paper's own configuration: cell measurements by its rule (Section III-A) and its
    stop rule, against the EXACT rule (equal to brute force) on the same index.  Reports
    the share of queries whose PAPER neighbours differ (misses) and predictions differ."""
    prob = W.make(args.workload)
    dev = torch.device("cuda:0")
    if prob.dtype == "bf16":
        pts = torch.from_numpy(prob.points.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        pts = torch.from_numpy(prob.points).to(dev)
    tgt = torch.from_numpy(prob.targets).to(dev)
    qs = torch.from_numpy(prob.queries).to(dev)
    t0 = time.perf_counter()
    w, o, splits = ghn.ghn_cell_measure(pts)
    measure_ms = (time.perf_counter() - t0) * 1e3
    rows = []
    for label, widths, origin in (("paper_rule_widths", w, o), ("about_8_per_cell", prob.cell_width, None)):
        print("paper study: %s grid" % label, file=sys.stderr, flush=True)
        if label == "paper_rule_widths" and int(splits.max()) > 4096:
            # a query in a sparse region walks about (neighbour radius / finest width) layers
            rows.append({"grid": label, "skipped": "the rule gives %d splits in a dimension (width %.3g); queries in "
                         "sparse regions would walk thousands of layers" % (int(splits.max()), float(w.min()))})
            continue
        try:
            ix = ghn.Index(pts, tgt, prob.task, widths, origin)
        except ghn.GHNError as e:  # e.g. cell ids too wide for the 64-bit Morton key of the tree
            rows.append({"grid": label, "build_error": str(e)})
            continue
        res = {}
        for name, stop in (("exact", ghn.GHN_STOP_EXACT), ("paper", ghn.GHN_STOP_PAPER)):
            ix.predict(qs, prob.k, stop=stop, with_d2=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ix.predict(qs, prob.k, stop=stop, with_d2=False, with_stats=True)
            torch.cuda.synchronize()
            res[name] = dict(ms=(time.perf_counter() - t0) * 1e3, idx=r["idx"], pred=r["pred"],
                             layers=float(r["stop_layer"].double().mean().item()),
                             cands=float(r["cands"].double().mean().item()))
        same_set = (torch.sort(res["paper"]["idx"], dim=1)[0] == torch.sort(res["exact"]["idx"], dim=1)[0]).all(1)
        rows.append({"grid": label, "num_cells": int(ix.info.num_cells),
                     "query_miss_rate": float(1.0 - same_set.double().mean().item()),
                     "prediction_differs_rate": float((res["paper"]["pred"] != res["exact"]["pred"]).double()
                                                      .mean().item()),
                     "exact_ms": res["exact"]["ms"], "paper_ms": res["paper"]["ms"],
                     "exact_mean_layers": res["exact"]["layers"], "paper_mean_layers": res["paper"]["layers"],
                     "exact_cands_per_query": res["exact"]["cands"], "paper_cands_per_query": res["paper"]["cands"]})
        ix.close()
    print(json.dumps({"study": "PAPER stop rule vs EXACT (= brute force)", "workload": describe(prob, "both"),
                      "cell_measure_ms": measure_ms, "paper_rule_splits": [int(x) for x in splits],
                      "paper_rule_widths": [float(x) for x in w], "grids": rows}), flush=True)


def cpu_more(prob, target_s: float = 5.0):
    """More CPU figures of the oracle: the grid walk on one thread and exhaustive KNN on all
    threads, each on a bounded query sample, plus the host description."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    out = {"host": {"nproc": os.cpu_count(), "omp_threads": threads, "cpu_model": model}}

    def timed(fn, pilot):
        t0 = time.perf_counter()
        fn(pilot)
        dt = time.perf_counter() - t0
        count = int(min(prob.m, max(pilot, pilot * target_s / max(dt, 1e-6))))
        t0 = time.perf_counter()
        fn(count)
        return count, time.perf_counter() - t0

    g = oracle.Grid(prob.points_f32(), prob.targets, prob.task, prob.cell_width)
    c, dt = timed(lambda c: g.predict(prob.queries[:c], prob.k, oracle.STOP_EXACT, nthreads=1), 8)
    g.close()
    out["grid_1_thread"] = {"value": c / dt, "unit": "queries/s", "sample": "first %d queries" % c}
    pts = prob.points_f32()
    c, dt = timed(lambda c: oracle.bruteforce(pts, prob.targets, prob.task, prob.queries[:c], prob.k,
                                              nthreads=threads), max(threads, 4))
    out["bruteforce_all_threads"] = {"value": c / dt, "unit": "queries/s", "threads": threads,
                                     "sample": "first %d queries" % c}
    return out


def bench_multi(args, ghn, W, torch):
    """Many independent 3-D problems: per-index launches vs one batched launch (and its graph replay)."""
    probs = W.make_multi3d()
    dev = torch.device("cuda:0")
    stop = ghn.GHN_STOP_EXACT if args.stop == "exact" else ghn.GHN_STOP_PAPER
    # FP32 forms, EXACT rule: the central cell and layer 1 in one ring step (batched input
    # order 4.01 -> 3.21 ms); the neighbours do not depend on it
    ring = args.ring_step if args.ring_step >= 0 else (2 if stop == ghn.GHN_STOP_EXACT else 0)
    t0 = time.perf_counter()
    idxs, qs, outs = [], [], []
    for p in probs:
        ix = ghn.Index(torch.from_numpy(p.points).to(dev), torch.from_numpy(p.targets).to(dev), p.task, p.cell_width)
        idxs.append(ix)
        qs.append(torch.from_numpy(p.queries).to(dev))
        outs.append((torch.empty((p.m, p.k), dtype=torch.int64, device=dev),
                     torch.empty(p.m, dtype=torch.int32, device=dev)))
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    M = sum(p.m for p in probs)
    f = 3
    # work counts (untimed)
    cands = probes = 0
    alg_bytes = ext_bytes = 0
    for p, ix, q in zip(probs, idxs, qs):
        st = ix.predict(q, p.k, stop=stop, with_d2=False, with_stats=True, ring_step=ring)
        c, pr = int(st["cands"].sum().item()), int(st["probes"].sum().item())
        cands += c
        probes += pr
        alg_bytes += walk_bytes(p.m, f, p.k, c, pr)
        ext_bytes += walk_bytes_extended(p.m, f, p.k, c, pr)
    torch.cuda.synchronize()

    def timeit(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        ev[0].record()
        for i in range(args.steps):
            step()
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
        return float(ev[0].elapsed_time(ev[-1])) / args.steps, per

    forms = {}
    if "fp32" in args.forms:
        def per_item():
            for p, ix, q, (oi, op) in zip(probs, idxs, qs, outs):
                ghn.ghn_predict(ix.handle, q, p.k, oi, op, None, stop, ghn.GHN_PREC_FP32, ghn.GHN_FLAG_NO_SORT,
                                ring_step=ring)
        ms, per = timeit(per_item)
        forms["fp32_per_index"] = dict(ms=ms, per=per)
        items = [(ix.handle, q, p.k, oi, op, None) for p, ix, q, (oi, op) in zip(probs, idxs, qs, outs)]
        # input order (items one after another) and spatial order (sorted by item and cell)
        wsi = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, stop, ghn.GHN_PREC_FP32, ghn.GHN_FLAG_NO_SORT),
                          dtype=torch.uint8, device=dev)
        batch_in = ghn.ghn_batch_prepare(items, wsi, stop=stop, flags=ghn.GHN_FLAG_NO_SORT, ring_step=ring)
        ms, per = timeit(lambda: ghn.ghn_predict_batched(batch_in))
        forms["fp32_batched_input_order"] = dict(ms=ms, per=per)
        ws = torch.empty(ghn.ghn_batch_workspace_bytes_for(items, stop), dtype=torch.uint8, device=dev)
        batch = ghn.ghn_batch_prepare(items, ws, stop=stop, ring_step=ring)
        ms, per = timeit(lambda: ghn.ghn_predict_batched(batch))
        forms["fp32_batched"] = dict(ms=ms, per=per)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                ghn.ghn_predict_batched(batch)
        torch.cuda.current_stream().wait_stream(side)
        ms, per = timeit(g.replay)
        forms["fp32_batched_graph"] = dict(ms=ms, per=per)
    if "bf16" in args.forms:
        wss = [torch.empty(max(ghn.ghn_predict_workspace_bytes(ix.handle, p.m, p.k, stop, ghn.GHN_PREC_BF16_MFMA, 0,
                                                               args.group_levels), 1),
                           dtype=torch.uint8, device=dev) for p, ix in zip(probs, idxs)]

        def per_item16():
            for p, ix, q, (oi, op), w in zip(probs, idxs, qs, outs, wss):
                ghn.ghn_predict(ix.handle, q, p.k, oi, op, None, stop, ghn.GHN_PREC_BF16_MFMA, 0, ws=w,
                                group_levels=args.group_levels)
        ms, per = timeit(per_item16)
        forms["bf16_per_index"] = dict(ms=ms, per=per)
        # the same grouped launches, all captured in one graph and replayed as one launch
        g16 = torch.cuda.CUDAGraph()
        side16 = torch.cuda.Stream()
        side16.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side16):
            with torch.cuda.graph(g16, stream=side16):
                per_item16()
        torch.cuda.current_stream().wait_stream(side16)
        ms, per = timeit(g16.replay)
        forms["bf16_per_index_graph"] = dict(ms=ms, per=per)
        # all items' query groups in one grouped persistent launch (one sort of every
        # query by (item, cell), then one walk kernel), and its graph replay
        items16 = [(ix.handle, q, p.k, oi, op, None) for p, ix, q, (oi, op) in zip(probs, idxs, qs, outs)]
        ws16 = torch.empty(ghn.ghn_batch_workspace_bytes_for(items16, stop, ghn.GHN_PREC_BF16_MFMA, 0,
                                                             args.group_levels), dtype=torch.uint8, device=dev)
        batch16 = ghn.ghn_batch_prepare(items16, ws16, stop=stop, prec=ghn.GHN_PREC_BF16_MFMA,
                                        group_levels=args.group_levels)
        ms, per = timeit(lambda: ghn.ghn_predict_batched(batch16))
        forms["bf16_batched"] = dict(ms=ms, per=per)
        gb = torch.cuda.CUDAGraph()
        sideb = torch.cuda.Stream()
        sideb.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(sideb):
            with torch.cuda.graph(gb, stream=sideb):
                ghn.ghn_predict_batched(batch16)
        torch.cuda.current_stream().wait_stream(sideb)
        ms, per = timeit(gb.replay)
        forms["bf16_batched_graph"] = dict(ms=ms, per=per)
    best = min(forms, key=lambda n: forms[n]["ms"])
    B = forms[best]
    line = {
        "metric": METRIC, "value": M / (B["ms"] * 1e-3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": B["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if best.startswith("fp32") else "bf16+f32+f64", "data": "synthetic",
        "config": {"workload": "multi3d: %d independent uniform 3-D problems, n log-uniform in [1e3, 2e6] (sum %d), "
                               "sum m = %d queries, k in {1,5,10,20}, majority vote, %s stop" % (
                                   len(probs), sum(p.n for p in probs), M, args.stop.upper()),
                   "problems": len(probs), "sum_n": sum(p.n for p in probs), "sum_m": M, "form": best,
                   "fp32_ring_step": ring},
        "roofline": hbm_roofline(alg_bytes, ext_bytes, B["ms"],
                                 measured_traffic("multi3d", "fp32_batched") if best.startswith("fp32_batched")
                                 else None,
                                 "k_predict_batched" if "batched" in best else "per-index kernels"),
        "forms": {n: {"qps": M / (v["ms"] * 1e-3), "ms_per_step": v["ms"],
                      "step_ms_p10_p50_p90": [float(np.percentile(v["per"], 10)), float(np.median(v["per"])),
                                              float(np.percentile(v["per"], 90))]} for n, v in forms.items()},
        "work": {"candidates_per_query": cands / M, "index_reads_per_query": probes / M,
                 "algorithmic_bytes_per_step": alg_bytes},
        "build_ms": build_ms,
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        done_q, t_cpu, used = 0, 0.0, 0
        for p in probs[::8]:
            g = oracle.Grid(p.points, p.targets, p.task, p.cell_width)
            t1 = time.perf_counter()
            g.predict(p.queries, p.k, oracle.STOP_EXACT, nthreads=threads)
            t_cpu += time.perf_counter() - t1
            done_q += p.m
            used += 1
            g.close()
            if t_cpu > 15.0:
                break
        line["cpu_baseline"] = {"value": done_q / t_cpu, "unit": "queries/s", "cores": threads, "kind": "oracle",
                                "sample": "all queries of %d of the %d problems (every 8th), grid walk with EXACT "
                                          "stop, FP64, OpenMP over queries" % (used, len(probs))}
    print(json.dumps(line), flush=True)


def query_parts(prob, qs, ix, ghn, torch, stop, sort32, levels16, reps=3, ring32=0, grow32=0, gs16=0, tw16=0):
    """Each half of a mixed query set (cluster / uniform background) timed on its own, both forms."""
    out = {}
    k = prob.k
    for name, val in (("cluster", 1), ("uniform", 0)):
        sel = torch.from_numpy(np.nonzero(prob.query_part == val)[0]).to(qs.device)
        q = qs.index_select(0, sel).contiguous()
        mq = int(q.shape[0])
        if mq == 0:
            continue
        oi = torch.empty((mq, k), dtype=torch.int64, device=qs.device)
        op = torch.empty(mq, dtype=torch.int32 if prob.task == 0 else torch.float32, device=qs.device)
        part = {"queries": mq}
        for form, prec, flags, levels, ring, gs, tw in (
                ("fp32_plain", ghn.GHN_PREC_FP32, (0 if sort32 else ghn.GHN_FLAG_NO_SORT) | grow32, -1, ring32, 0, 0),
                ("bf16_grouped", ghn.GHN_PREC_BF16_MFMA, 0, levels16, 0, gs16, tw16)):
            nws = ghn.ghn_predict_workspace_bytes(ix.handle, mq, k, stop, prec, flags, levels)
            ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=qs.device)
            st = ix.predict(q, k, stop=stop, prec=prec, flags=flags, with_d2=False, with_stats=True,
                            group_levels=levels, ring_step=ring, group_size=gs, tile_width=tw)
            torch.cuda.synchronize()
            cands = float(st["cands"].double().mean().item())
            layers = float(st["stop_layer"].double().mean().item())
            del st
            ms = []
            for _ in range(reps + 1):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ghn.ghn_predict(ix.handle, q, k, oi, op, None, stop, prec, flags, ws=ws, group_levels=levels,
                                walk_events=(e0, e1), ring_step=ring, group_size=gs, tile_width=tw)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            kern = float(np.mean(ms[1:]))
            part[form] = {"kernel_ms": kern, "qps_kernel": mq / (kern * 1e-3), "candidates_per_query": cands,
                          "mean_stop_layer": layers}
        out[name] = part
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="clusters4d")
    ap.add_argument("--stop", default="exact", choices=["exact", "paper"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort", action="store_true", help="FP32 form: walk queries in spatial (Morton) order")
    ap.add_argument("--forms", default=None,
                    help="comma list of forms to time: fp32, bf16, persistent (GHN walks; persistent = the FP32 walk "
                         "through the batched persistent launch), brute (exhaustive KNN, reported beside); default "
                         "fp32,bf16, plus persistent for skew8d")
    ap.add_argument("--group-levels", type=int, default=-1, help="bf16 form: cell-id bits dropped to group queries")
    ap.add_argument("--group-size", type=int, default=0, help="bf16 form: most queries per group (0 = 16)")
    ap.add_argument("--tile-width", type=int, default=0, help="bf16 form: candidates per screened tile, 32 or 64 "
                                                               "(0 = 64)")
    ap.add_argument("--ring-step", type=int, default=-1,
                    help="FP32 form, EXACT rule: layers per step of the walk (-1: the autotuned value, else 2, so the "
                         "central cell and layer 1 are walked in one step; the neighbours do not depend on it)")
    ap.add_argument("--ring-grow", action="store_true",
                    help="FP32 form, EXACT rule: double the ring step while the buffer is not full (as the "
                         "autotuner may choose; for profiler runs of an autotuned configuration)")
    ap.add_argument("--autotune", choices=("auto", "on", "off"), default="auto",
                    help="pick the cell width (and each form's settings) with ghn_autotune on a query sample "
                         "before the timed region; auto = on for %s" % ", ".join(AUTOTUNED))
    ap.add_argument("--tune-queries", type=int, default=32768, help="query sample size for --autotune")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the forms only: no autotuning and no per-half runs (for profiler runs, so the "
                         "walk kernels' dispatches are all of the timed configuration)")
    ap.add_argument("--lookup", choices=("auto", "dense", "tree", "hash"), default="auto",
                    help="cell lookup to build (default: the build's choice, or the autotuned one)")
    ap.add_argument("--cell-width", type=float, default=None,
                    help="cell width to build with (default: the workload's calibrated width, or the autotuned one)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--paper-study", action="store_true",
                    help="instead of the benchmark: the paper's cell measurements and stop rule against EXACT")
    ap.add_argument("--write-traffic", metavar="PMC_DIR",
                    help="no GPU work: write profiles/traffic.json from rocprofv3 --pmc output for --workload "
                         "(a comma list)")
    args = ap.parse_args()
    if args.forms is None:
        args.forms = "fp32,bf16" + (",persistent" if args.workload == "skew8d" else "")
    if args.write_traffic:
        write_traffic(args.write_traffic, args.workload.split(","), args=args)
        return
    if args.gpus != 1:
        print("bench.py: this benchmark measures one GPU only; run with --gpus 1", file=sys.stderr)
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

    if args.workload == "multi3d":
        bench_multi(args, ghn, W, torch)
        return
    if args.paper_study:
        paper_study(args, ghn, W, torch)
        return
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

    m, k = prob.m, prob.k
    f = prob.f
    width = prob.cell_width if args.cell_width is None else args.cell_width
    lookup = {"auto": None, "dense": ghn.GHN_LOOKUP_DENSE, "tree": ghn.GHN_LOOKUP_TREE,
              "hash": ghn.GHN_LOOKUP_HASH}[args.lookup]
    tuned = None
    sort32, levels16 = args.sort, args.group_levels
    ring32, grow32 = 0, 0  # FP32 form: the EXACT walk's ring schedule (autotuned, else --ring-step)
    gs16 = args.group_size  # bf16 form: most queries per group (autotuned; 0 = 16)
    tw16 = args.tile_width  # bf16 form: candidates per screened tile (autotuned; 0 = 64)
    if args.autotune == "on" or (args.autotune == "auto" and args.workload in AUTOTUNED and args.cell_width is None
                                    and not args.no_extras):
        # widths around the calibrated one (under PAPER only execution settings are tuned);
        # the chosen width is the fastest setting's, then each form takes its own best trial there
        widths = [prob.cell_width] if stop == ghn.GHN_STOP_PAPER else \
            [prob.cell_width * 2.0 ** (i / 2.0) for i in range(-2, 5)]
        ns = min(m, args.tune_queries)
        print("autotune: %d widths on %d queries" % (len(widths), ns), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        best, trials = ghn.ghn_autotune(pts, tgt, prob.task, qs[:ns], k, stop, widths)
        torch.cuda.synchronize()
        tune_ms = (time.perf_counter() - t0) * 1e3
        width = float(best["cell_width"])
        if best["lookup"] == ghn.GHN_LOOKUP_HASH:
            lookup = ghn.GHN_LOOKUP_HASH
        # FP32 trials of the lookup that will be built (the bf16 trials walk the tree either way)
        at_w = [t for t in trials if t["cell_width"] == best["cell_width"] and t["ms"] >= 0
                and (t["prec"] != ghn.GHN_PREC_FP32
                     or (t["lookup"] == ghn.GHN_LOOKUP_HASH) == (lookup == ghn.GHN_LOOKUP_HASH))]
        b32 = min((t for t in at_w if t["prec"] == ghn.GHN_PREC_FP32), key=lambda t: t["ms"], default=None)
        b16 = min((t for t in at_w if t["prec"] == ghn.GHN_PREC_BF16_MFMA), key=lambda t: t["ms"], default=None)
        if b32 is not None:
            sort32 = not (b32["flags"] & ghn.GHN_FLAG_NO_SORT)
            ring32 = int(b32["ring_step"])
            grow32 = int(b32["flags"]) & ghn.GHN_FLAG_RING_GROW
        if b16 is not None:
            levels16 = int(b16["group_levels"])
            gs16 = int(b16["group_size"])
            tw16 = int(b16["tile_width"])
        tuned = {"cell_width": width, "tune_ms": tune_ms, "sample_queries": ns, "widths_tried": widths,
                 "fp32_sort": sort32, "fp32_ring_step": ring32, "fp32_ring_grow": bool(grow32),
                 "bf16_group_levels": levels16, "bf16_group_size": gs16, "bf16_tile_width": tw16,
                 "trials": [{"w": t["cell_width"], "prec": "fp32" if t["prec"] == ghn.GHN_PREC_FP32 else "bf16",
                             "lookup": t["lookup"], "levels": t["group_levels"], "flags": t["flags"],
                             "ring_step": t["ring_step"], "group_size": t["group_size"],
                             "tile_width": t["tile_width"], "ms": t["ms"]}
                            for t in trials]}
        print("autotune: width %.6g (calibrated %.6g), %.1f s" % (width, prob.cell_width, tune_ms * 1e-3),
              file=sys.stderr, flush=True)
    if args.ring_grow:
        grow32 = ghn.GHN_FLAG_RING_GROW
    if args.ring_step >= 0:
        ring32 = args.ring_step
    elif tuned is None and stop == ghn.GHN_STOP_EXACT:
        # layers 0 and 1 in one step: the central cell alone rarely fills the buffer, so its own
        # pass (run list, stop test) buys no pruning (clusters4d walk 0.348 -> 0.331 ms)
        ring32 = 2

    t0 = time.perf_counter()
    ix = ghn.Index(pts, tgt, prob.task, width, lookup=lookup)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    out_idx = torch.empty((m, k), dtype=torch.int64, device=dev)
    out_pred = torch.empty(m, dtype=torch.int32 if prob.task == 0 else torch.float32, device=dev)

    def timed(step):
        """Warm up, then time `steps` back-to-back calls between two events; each call also
        gets a (begin, end) event pair that the library records around its walk kernel on
        the same stream.  Per-step times are the spacings of the walk-begin events."""
        for _ in range(args.warmup):
            step(None)
        torch.cuda.synchronize()
        mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        wb, we = mk(), mk()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for i in range(args.steps):
            step((wb[i], we[i]))
        end.record()
        torch.cuda.synchronize()
        ms = float(start.elapsed_time(end)) / args.steps
        per = np.array([wb[i].elapsed_time(wb[i + 1]) for i in range(args.steps - 1)] + [wb[-1].elapsed_time(end)])
        kern = np.array([wb[i].elapsed_time(we[i]) for i in range(args.steps)])
        return ms, float(kern.mean()), per

    def stats(prec, flags=0, levels=-1, ring=0, gsize=0, tw=0):
        st = ix.predict(qs, k, stop=stop, prec=prec, flags=flags, with_d2=False, with_stats=True, group_levels=levels,
                        ring_step=ring, group_size=gsize, tile_width=tw)
        torch.cuda.synchronize()
        out = dict(cands=int(st["cands"].sum().item()), probes=int(st["probes"].sum().item()),
                   layers=float(st["stop_layer"].double().mean().item()),
                   rerank=float(st["rerank"].double().mean().item()))
        del st
        return out

    # this run's settings, matched against those the committed counter runs were taken with
    run32 = {"cell_width": width, "ring_step": ring32, "ring_grow": bool(grow32), "sort": bool(sort32)}
    run16 = {"cell_width": width, "group_levels": levels16, "group_size": gs16 or 16, "tile_width": tw16 or 64}
    forms = {}
    if "fp32" in args.forms:
        # per-query walk; with --sort a step = spatial order (Morton sort) + walk, events
        # between the two calls time the walk kernel alone on the stream both run on
        flags = (0 if sort32 else ghn.GHN_FLAG_NO_SORT) | grow32
        w = stats(ghn.GHN_PREC_FP32, flags, ring=ring32)
        order = torch.empty(m, dtype=torch.int32, device=dev)
        ows = torch.empty(max(ghn.ghn_query_order_workspace_bytes(m), 1), dtype=torch.uint8, device=dev)

        def step32(evs):
            if sort32:
                ghn.ghn_query_order(ix.handle, qs, order, ows)
                ghn.ghn_predict(ix.handle, qs, k, out_idx, out_pred, None, stop, ghn.GHN_PREC_FP32, grow32,
                                order=order, walk_events=evs, ring_step=ring32)
            else:
                ghn.ghn_predict(ix.handle, qs, k, out_idx, out_pred, None, stop, ghn.GHN_PREC_FP32, flags,
                                walk_events=evs, ring_step=ring32)

        ms, kern_ms, per = timed(step32)
        alg_bytes = walk_bytes(m, f, k, w["cands"], w["probes"])
        forms["fp32_plain"] = dict(
            qps=m / (ms * 1e-3), ms_per_step=ms, kernel_ms=kern_ms, per=per, work=w,
            roofline=hbm_roofline(alg_bytes, walk_bytes_extended(m, f, k, w["cands"], w["probes"]), kern_ms,
                                  measured_traffic(args.workload, "fp32", run32, prob.cell_width),
                                  "k_predict_%s" % ("tree" if ix.info.lookup == 1 else "dense")),
            alg={"bytes_per_step": alg_bytes})
    if "bf16" in args.forms:
        nws = ghn.ghn_predict_workspace_bytes(ix.handle, m, k, stop, ghn.GHN_PREC_BF16_MFMA, 0, levels16)
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
        w = stats(ghn.GHN_PREC_BF16_MFMA, 0, levels16, gsize=gs16, tw=tw16)

        def step16(evs):
            ghn.ghn_predict(ix.handle, qs, k, out_idx, out_pred, None, stop, ghn.GHN_PREC_BF16_MFMA, 0, ws=ws,
                            group_levels=levels16, walk_events=evs, group_size=gs16, tile_width=tw16)

        ms, kern_ms, per = timed(step16)
        flops = 2.0 * f * w["cands"]  # algorithmic: 2 f per screened (query, candidate) pair
        achieved = flops / (kern_ms * 1e-3) / 1e12
        forms["bf16_grouped"] = dict(
            qps=m / (ms * 1e-3), ms_per_step=ms, kernel_ms=kern_ms, per=per, work=w,
            roofline={"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": measured_traffic(args.workload, "bf16", run16, prob.cell_width),
                      "kernel": "k_predict_group"},
            alg={"flops_per_step": flops, "issued_mfma_flops_per_step": 2.0 * (-(-3 * f // 32) * 32) * w["cands"]})
        # the screen's distance error against FP64, on a query sample against points spread over the index
        ns = min(m, 2048)
        ea, er = ghn.ghn_screen_error(ix.handle, qs[:ns], sample=8192)
        forms["bf16_grouped"]["screen_error"] = {
            "max_abs": float(ea.max().item()), "max_rel": float(er.max().item()), "mean_rel": float(er.mean().item()),
            "bound_rel": 2.0 ** -13.8, "admission_margin_rel": 2.0 ** -12,
            "sample": "first %d queries x %d points spread over the index; rel = |s - d| / (|q'|^2 + |x'|^2)"
                      % (ns, min(8192, prob.n))}

    if "persistent" in args.forms:
        # the same FP32 walk through the batched persistent launch (waves take queries from
        # 8 per-XCD ranges of atomic counters until none are left), in the spatial order
        # the FP32 form uses (the launch then sorts the queries first)
        pflags = (0 if sort32 else ghn.GHN_FLAG_NO_SORT) | grow32
        w = stats(ghn.GHN_PREC_FP32, pflags, ring=ring32)
        pitems = [(ix.handle, qs, k, out_idx, out_pred, None)]
        bws = torch.empty(max(ghn.ghn_batch_workspace_bytes_for(pitems, stop, ghn.GHN_PREC_FP32, pflags), 1),
                          dtype=torch.uint8, device=dev)
        batch = ghn.ghn_batch_prepare(pitems, bws, stop, flags=pflags, ring_step=ring32)

        def stepp(evs):
            if evs:
                evs[0].record()
            ghn.ghn_predict_batched(batch)
            if evs:
                evs[1].record()

        ms, kern_ms, per = timed(stepp)
        ghn.ghn_batch_destroy(batch)
        alg_bytes = walk_bytes(m, f, k, w["cands"], w["probes"])
        forms["fp32_persistent"] = dict(
            qps=m / (ms * 1e-3), ms_per_step=ms, kernel_ms=kern_ms, per=per, work=w,
            roofline=hbm_roofline(alg_bytes, walk_bytes_extended(m, f, k, w["cands"], w["probes"]), kern_ms,
                                  measured_traffic(args.workload, "fp32_batched", run32, prob.cell_width),
                                  "k_predict_batched"),
            alg={"bytes_per_step": alg_bytes, "timed": "counter reset (+ query sort) + persistent kernel",
                 "spatial_order": bool(sort32)})
    if "brute" in args.forms:
        # exhaustive KNN (the paper's comparison method) on the same GPU and index data
        nws = ghn.ghn_predict_workspace_bytes(ix.handle, m, k, stop, ghn.GHN_PREC_BF16_MFMA, 0)
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)

        def stepb(evs):
            ghn.ghn_bruteforce(ix.handle, qs, k, out_idx, out_pred, None, 0, None, ws, walk_events=evs)

        ms, kern_ms, per = timed(stepb)
        pairs = float(m) * float(prob.n)
        flops = 2.0 * f * pairs
        achieved = flops / (kern_ms * 1e-3) / 1e12
        forms["bruteforce_bf16"] = dict(
            qps=m / (ms * 1e-3), ms_per_step=ms, kernel_ms=kern_ms, per=per,
            work=dict(cands=pairs, probes=0, layers=0.0),
            roofline={"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": None, "kernel": "k_predict_group"},
            alg={"flops_per_step": flops})
    for v in forms.values():
        r = v["roofline"]
        if r["unit"] == "GB/s" and r["frac"] > 1.0:
            r["note"] = ("algorithmic bytes count every candidate gather; above the HBM peak, repeated candidates "
                         "of nearby queries were served from L2 and the Infinity Cache (traffic is the HBM-side count)")
    walk_forms = [name for name in forms if name != "bruteforce_bf16"]
    best = max(walk_forms, key=lambda name: forms[name]["qps"])
    B = forms[best]
    line = {
        "metric": METRIC,
        "value": B["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": B["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if best.startswith("fp32") else "bf16+f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(prob, args.stop.upper()), "n": prob.n, "f": f, "m": m, "k": k,
                   "cell_width": width, "stop": args.stop, "form": best,
                   "lookup": {0: "dense", 1: "tree", 2: "hash"}[ix.info.lookup],
                   "fp32_ring_step": ring32, "fp32_ring_grow": bool(grow32), "fp32_sorted": bool(sort32)},
        "roofline": B["roofline"],
        "forms": {name: {"qps": v["qps"], "ms_per_step": v["ms_per_step"], "kernel_ms": v["kernel_ms"],
                         "step_ms_p10_p50_p90": [float(np.percentile(v["per"], 10)), float(np.median(v["per"])),
                                                 float(np.percentile(v["per"], 90))],
                         "candidates_per_query": v["work"]["cands"] / m, "index_reads_per_query": v["work"]["probes"] / m,
                         "mean_stop_layer": v["work"]["layers"], "rerank_per_query": v["work"].get("rerank"),
                         "roofline": v["roofline"], "algorithmic": v["alg"],
                         **({"screen_error": v["screen_error"]} if "screen_error" in v else {})}
                  for name, v in forms.items()},
        "build_ms": build_ms,
        "index": {"num_cells": int(ix.info.num_cells), "box_cells": int(ix.info.box_cells),
                  "max_occupancy": int(ix.info.max_occupancy)},
    }
    if tuned is not None:
        line["config"]["cell_width_source"] = "autotuned"
        line["autotune"] = tuned
    if prob.query_part is not None and not args.no_extras:
        line["query_parts"] = query_parts(prob, qs, ix, ghn, torch, stop, sort32, levels16, ring32=ring32,
                                          grow32=grow32, gs16=gs16, tw16=tw16)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
        line["cpu_oracle_more"] = cpu_more(prob)
    ix.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
