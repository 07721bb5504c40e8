"""Find, per workload, the scalar cell width that gives ~8 training points per occupied cell.

Uses only the oracle's occupied-cell count (Eq. 1 + Algorithm 1) and a bisection
on log(width).  The printed widths are the `width` entries of the workload table
in paper_2004_02290_amd/workloads.py.

    python -m oracle.calibrate_widths blobs2d clusters4d
"""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle
from paper_2004_02290_amd import workloads as W


def calibrate(points: np.ndarray, target: float = 8.0, rel_tol: float = 0.01, iters: int = 40) -> float:
    n = points.shape[0]
    lo, hi = 1e-4, 4.0
    for _ in range(iters):
        mid = float(np.float32(math.exp(0.5 * (math.log(lo) + math.log(hi)))))
        per_cell = n / oracle.count_cells(points, mid)
        if abs(per_cell / target - 1.0) <= rel_tol:
            return mid
        if per_cell < target:
            lo = mid
        else:
            hi = mid
    return mid


def main(names):
    for name in names:
        prob = W.make(name)
        w = calibrate(prob.points_f32())
        cells = oracle.count_cells(prob.points_f32(), w)
        print(f"{name}: width={w:.8g} cells={cells} points/cell={prob.n / cells:.3f}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(W.WORKLOADS))
