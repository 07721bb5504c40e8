"""Autotuning driver: runs ghn_autotune on a query sample and caches the choice.

The cache is a JSON file keyed by (n, f, dtype, k, stop rule, a coarse data
signature: per-dimension coordinate range of a point sample); it stores the
chosen cell width, screen, grouping and flags.  Under the EXACT stop rule the
choice never changes the neighbours returned (every width gives brute-force
results); under the PAPER rule only execution settings are tuned.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import numpy as np
import torch

from . import binding as ghn


def signature(points: torch.Tensor, k: int, stop: int) -> str:
    n, f = points.shape
    sample = points[:: max(1, n // 4096)].float()
    lo = sample.min(dim=0).values.cpu().numpy()
    hi = sample.max(dim=0).values.cpu().numpy()
    rng = ",".join("%.3g:%.3g" % (a, b) for a, b in zip(lo, hi))
    return "n=%d f=%d dtype=%s k=%d stop=%d range=%s" % (n, f, str(points.dtype), k, stop, rng)


def tune(points: torch.Tensor, targets: torch.Tensor, task: int, query_sample: torch.Tensor, k: int,
         stop: int = ghn.GHN_STOP_EXACT, widths=None, cache_path: Optional[str] = None):
    """Return the best setting (dict with cell_width, lookup, prec, group_levels, flags, ms)."""
    key = signature(points, k, stop)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            return cache[key]
    best, trials = ghn.ghn_autotune(points, targets, task, query_sample, k, stop, widths)
    best = {name: (float(v) if isinstance(v, (float, np.floating)) else int(v)) for name, v in best.items()}
    best["trials"] = trials
    if cache_path:
        cache[key] = best
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return best
