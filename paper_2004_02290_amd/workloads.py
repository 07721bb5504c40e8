"""Seeded synthetic inputs shaped like the workloads the GHN paper evaluates on.

The paper (Section IV, Table 1) measures on public datasets that were scaled and
reduced by PCA to a few dimensions, then split 80/20 into training points and
queries.  None of those datasets is available here, so each workload below is a
seeded stand-in with the same structure: low-dimensional, class-labelled (or a
smooth regression target), with dense cluster cores and sparse tails.

This module only draws random numbers.  It holds none of the method's
arithmetic (no cell hashing, no distances, no selection), so both the GPU
library and the CPU oracle can take their inputs from it.

Every workload uses ``numpy.random.default_rng`` (PCG64) streams spawned from
``SeedSequence(seed)`` in a fixed order, so a (name, n, m, seed) tuple always
produces the same arrays.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

CLASSIFY = 0
REGRESS = 1


@dataclasses.dataclass
class Problem:
    """One KNN problem: training points + targets, queries, k and a cell width."""
    name: str
    points: np.ndarray          # n x f, float32 (or uint16 bf16 bits when dtype == "bf16")
    targets: np.ndarray         # n int32 labels, or n float32 regression targets
    queries: np.ndarray         # m x f, float32
    k: int
    task: int                   # CLASSIFY or REGRESS
    cell_width: float           # scalar width used for every dimension
    dtype: str = "f32"          # storage type of `points`: "f32" or "bf16"
    query_part: Optional[np.ndarray] = None  # per query: 1 drawn from a cluster, 0 from the uniform background

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def m(self) -> int:
        return int(self.queries.shape[0])

    @property
    def f(self) -> int:
        return int(self.points.shape[1])

    def points_f32(self) -> np.ndarray:
        """Points as float32 (bf16 bits are widened exactly)."""
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.points)
        return self.points


# --------------------------------------------------------------------------------------
# Workload table.  Sizes, spreads, label counts and k follow the configurations the
# benchmark is quoted on; `width` is the scalar cell width at the full size that gives
# about 8 training points per occupied cell.  The widths were found by bisection on
# the oracle's occupied-cell count (oracle/calibrate_widths.py writes them).
# --------------------------------------------------------------------------------------
WORKLOADS: Dict[str, dict] = {
    # 3 isotropic Gaussian blobs in 2-D, labels = blob id.
    "blobs2d": dict(f=2, n=10_000, m=1_000, k=5, task=CLASSIFY, seed=1,
                    centers=3, sigma=0.1, width=0.021281155),
    # 10 Gaussian clusters in 4-D, 10 classes.  The headline workload.
    "clusters4d": dict(f=4, n=1_000_000, m=100_000, k=10, task=CLASSIFY, seed=2,
                       centers=10, sigma=0.05, width=0.023601368),
    # 5 tight clusters + 10% uniform background in 8-D, regression target.
    "skew8d": dict(f=8, n=10_000_000, m=1_000_000, k=16, task=REGRESS, seed=3,
                   centers=5, sigma=0.02, width=0.031533688),
    # 32 clusters in 16-D, points stored as bf16, 32 classes.
    "bf16_16d": dict(f=16, n=4_000_000, m=500_000, k=32, task=CLASSIFY, seed=4,
                     centers=32, sigma=0.03, width=0.11001434),
}

# Many independent uniform 3-D problems of log-uniform size.
MULTI3D = dict(f=3, problems=256, n_lo=1_000, n_hi=2_000_000, m_lo=1, m_hi=65_536,
               ks=(1, 5, 10, 20), labels=4, seed=5, per_cell=8.0)


def _streams(seed: int, count: int) -> List[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(count)]


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even); returns uint16 bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = ((u >> np.uint64(16)) & np.uint64(1)) + np.uint64(0x7FFF)
    return ((u + rounding) >> np.uint64(16)).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bits to float32 (exact)."""
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def _mixture(rng_lab, rng_noise, centers: np.ndarray, sigma: float, count: int):
    lab = rng_lab.integers(0, centers.shape[0], size=count)
    x = centers[lab] + rng_noise.normal(0.0, sigma, size=(count, centers.shape[1]))
    return x.astype(np.float32), lab.astype(np.int32)


def make(name: str, n: Optional[int] = None, m: Optional[int] = None,
         seed: Optional[int] = None) -> Problem:
    """Generate workload `name`, optionally shrunk to n points / m queries.

    When shrunk, the cell width is scaled by (n_full / n) ** (1 / f) so that the
    number of points per occupied cell stays about the same.
    """
    w = WORKLOADS[name]
    f = w["f"]
    n_full, m_full = w["n"], w["m"]
    n = n_full if n is None else int(n)
    m = m_full if m is None else int(m)
    seed = w["seed"] if seed is None else int(seed)
    width = float(np.float32(w["width"] * (n_full / max(n, 1)) ** (1.0 / f)))

    if name in ("blobs2d", "clusters4d", "bf16_16d"):
        r_c, r_pl, r_pn, r_ql, r_qn = _streams(seed, 5)
        centers = r_c.random((w["centers"], f))
        pts, lab = _mixture(r_pl, r_pn, centers, w["sigma"], n)
        qs, _ = _mixture(r_ql, r_qn, centers, w["sigma"], m)
        if name == "bf16_16d":
            return Problem(name, f32_to_bf16_bits(pts), lab, qs, w["k"], CLASSIFY, width, "bf16")
        return Problem(name, pts, lab, qs, w["k"], CLASSIFY, width)

    if name == "skew8d":
        r_c, r_pa, r_pn, r_y, r_qa, r_qn = _streams(seed, 6)
        centers = r_c.random((w["centers"], f))
        pts, _ = _skewed(r_pa, r_pn, centers, w["sigma"], n, clustered_frac=0.9)
        y = np.sin(2.0 * np.pi * pts.astype(np.float64)).sum(axis=1)
        y = (y + r_y.normal(0.0, 0.01, size=n)).astype(np.float32)
        qs, part = _skewed(r_qa, r_qn, centers, w["sigma"], m, clustered_frac=0.5)
        return Problem(name, pts, y, qs, w["k"], REGRESS, width, query_part=part.astype(np.int8))

    raise KeyError(name)


def _skewed(r_assign, r_noise, centers, sigma, count, clustered_frac):
    """`clustered_frac` of the rows from the Gaussian clusters, the rest uniform on [0,1)^f.
    Returns the rows and, per row, whether it came from a cluster."""
    f = centers.shape[1]
    is_cluster = r_assign.random(count) < clustered_frac
    lab = r_assign.integers(0, centers.shape[0], size=count)
    x = np.empty((count, f), dtype=np.float32)
    nc = int(is_cluster.sum())
    x[is_cluster] = (centers[lab[is_cluster]] + r_noise.normal(0.0, sigma, size=(nc, f))).astype(np.float32)
    x[~is_cluster] = r_noise.random((count - nc, f)).astype(np.float32)
    return x, is_cluster


def make_multi3d(problems: Optional[int] = None, n_hi: Optional[int] = None,
                 m_hi: Optional[int] = None, seed: Optional[int] = None) -> List[Problem]:
    """Many independent uniform 3-D problems with log-uniform n and m.

    n_i = round(exp(U(ln n_lo, ln n_hi))), m_i = round(exp(U(ln 1, ln m_hi))),
    k_i uniform over {1, 5, 10, 20}, points and queries uniform on [0,1)^3 in
    float32 (so coordinates are multiples of 2^-24), labels uniform over 4
    classes.  Each cell width is (per_cell / n_i) ** (1/3): for uniform data the
    expected number of points per cell is then per_cell.
    """
    c = MULTI3D
    P = c["problems"] if problems is None else int(problems)
    n_hi = c["n_hi"] if n_hi is None else int(n_hi)
    m_hi = c["m_hi"] if m_hi is None else int(m_hi)
    seed = c["seed"] if seed is None else int(seed)
    r_sz, r_k, r_x, r_l, r_q = _streams(seed, 5)
    ns = np.rint(np.exp(r_sz.uniform(math.log(c["n_lo"]), math.log(n_hi), size=P))).astype(np.int64)
    ms = np.rint(np.exp(r_sz.uniform(0.0, math.log(m_hi), size=P))).astype(np.int64)
    ks = np.asarray(c["ks"])[r_k.integers(0, len(c["ks"]), size=P)]
    out = []
    for i in range(P):
        n_i, m_i = int(ns[i]), max(int(ms[i]), 1)
        k_i = int(min(ks[i], n_i))
        pts = r_x.random((n_i, 3), dtype=np.float32)
        lab = r_l.integers(0, c["labels"], size=n_i).astype(np.int32)
        qs = r_q.random((m_i, 3), dtype=np.float32)
        width = float(np.float32((c["per_cell"] / n_i) ** (1.0 / 3.0)))
        out.append(Problem(f"multi3d[{i}]", pts, lab, qs, k_i, CLASSIFY, width))
    return out


def lattice_problem(n: int, m: int, f: int, k: int, step: float = 0.25, span: int = 8,
                    seed: int = 0, task: int = CLASSIFY, width: float = 0.5,
                    labels: int = 3) -> Problem:
    """Points and queries on a coarse lattice: many exact distance ties and duplicates."""
    r_p, r_q, r_t = _streams(seed, 3)
    pts = (r_p.integers(-span, span + 1, size=(n, f)) * step).astype(np.float32)
    qs = (r_q.integers(-span - 2, span + 3, size=(m, f)) * step).astype(np.float32)
    if task == CLASSIFY:
        tgt = r_t.integers(0, labels, size=n).astype(np.int32)
    else:
        tgt = r_t.normal(0.0, 1.0, size=n).astype(np.float32)
    return Problem("lattice", pts, tgt, qs, k, task, float(np.float32(width)))


def uniform_problem(n: int, m: int, f: int, k: int, seed: int = 0, task: int = CLASSIFY,
                    width: float = 0.1, lo: float = 0.0, hi: float = 1.0, q_lo: Optional[float] = None,
                    q_hi: Optional[float] = None, labels: int = 4) -> Problem:
    """Uniform points on [lo, hi)^f; queries on [q_lo, q_hi)^f (defaults to the same box)."""
    r_p, r_q, r_t = _streams(seed, 3)
    q_lo = lo if q_lo is None else q_lo
    q_hi = hi if q_hi is None else q_hi
    pts = (lo + (hi - lo) * r_p.random((n, f))).astype(np.float32)
    qs = (q_lo + (q_hi - q_lo) * r_q.random((m, f))).astype(np.float32)
    if task == CLASSIFY:
        tgt = r_t.integers(0, labels, size=n).astype(np.int32)
    else:
        tgt = r_t.normal(0.0, 1.0, size=n).astype(np.float32)
    return Problem("uniform", pts, tgt, qs, k, task, float(np.float32(width)))
