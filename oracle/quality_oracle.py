"""CPU oracle of the decimation quality measures (test infrastructure only).

Sec. 6 judges a decimated cloud by how the number of neighbours of each
point grows with the neighbourhood's area: for points on a surface with a
uniform density the count grows linearly with the area.  For each radius
the paper plots the fractile bands (0.01-0.99, 0.1-0.9, 0.25-0.75) and the
mean of the per-point counts, fits a regression line of count against area
(its slope estimates the density) and reports R^2 and RMSE.  Eq. 2 states the
objective as the largest possible smallest distance between two kept
points, so the smallest nearest-neighbour distance is reported too.

Readings (the paper gives the measures, not their arithmetic):
* a neighbour of p within radius r is another point q with |p - q|^2 <= r^2,
  in exact integer arithmetic on int32 millimetre coordinates;
* fractile q of m counts is the element of rank floor(q (m - 1)) in
  ascending order (numpy's 'lower' quantile);
* the regression is ordinary least squares of count on area (m^2, pi r^2)
  over all (point, radius) pairs, computed from the exact integer sums of
  the counts and of their squares per radius.

Only tests/ call this module.  A library routine (scipy's cKDTree) finds the
candidate pairs; every distance is then checked exactly in integers.
"""
from __future__ import annotations

import math

import numpy as np

FRACTILES = (0.01, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99)


def neighbor_counts(P: np.ndarray, r2: list[int]) -> np.ndarray:
    """[m, R] uint32: other points within each squared radius r2 (mm^2)."""
    from scipy.spatial import cKDTree
    P = np.ascontiguousarray(P, dtype=np.int64)
    m, R = len(P), len(r2)
    out = np.zeros((m, R), dtype=np.uint32)
    if m == 0:
        return out
    tree = cKDTree(P.astype(np.float64))
    rmax = math.sqrt(max(r2)) + 1.0
    for i, nb in enumerate(tree.query_ball_point(P.astype(np.float64), rmax)):
        nb = np.asarray(nb, dtype=np.int64)
        nb = nb[nb != i]
        d2 = ((P[nb] - P[i]) ** 2).sum(axis=1)
        for r in range(R):
            out[i, r] = int((d2 <= r2[r]).sum())
    return out


def nn2(P: np.ndarray) -> np.ndarray:
    """[m] int64: squared distance from each point to its nearest other
    point (exact; candidates from the 4 nearest by the tree)."""
    from scipy.spatial import cKDTree
    P = np.ascontiguousarray(P, dtype=np.int64)
    m = len(P)
    tree = cKDTree(P.astype(np.float64))
    kq = min(m, 5)
    _, idx = tree.query(P.astype(np.float64), k=kq)
    idx = idx.reshape(m, kq)
    d2 = ((P[idx] - P[:, None, :]) ** 2).sum(axis=2)
    d2 = np.where(idx == np.arange(m)[:, None], np.iinfo(np.int64).max, d2)
    # points with more than 4 coincident copies: the nearest is at 0
    best = d2.min(axis=1)
    return best


def summary(counts: np.ndarray, r2: list[int], nn: np.ndarray | None = None) -> dict:
    """The measures of Sec. 6 from exact per-point counts [m, R]."""
    m, R = counts.shape
    area = [math.pi * v / 1e6 for v in r2]  # m^2
    S = [int(counts[:, r].astype(np.uint64).sum()) for r in range(R)]
    Q = [int((counts[:, r].astype(np.uint64) ** 2).sum()) for r in range(R)]
    fr = []
    for r in range(R):
        s = np.sort(counts[:, r])
        fr.append([int(s[int(math.floor(q * (m - 1)))]) for q in FRACTILES])
    n = m * R
    sx = m * sum(area)
    sxx = m * sum(a * a for a in area)
    sy = float(sum(S))
    syy = float(sum(Q))
    sxy = sum(a * s for a, s in zip(area, S))
    den = n * sxx - sx * sx
    slope = (n * sxy - sx * sy) / den if den != 0 else 0.0
    icpt = (sy - slope * sx) / n
    ss_res = syy - 2.0 * icpt * sy - 2.0 * slope * sxy + n * icpt * icpt + 2.0 * icpt * slope * sx + slope * slope * sxx
    ss_tot = syy - sy * sy / n
    r_sq = 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
    rmse = math.sqrt(max(ss_res, 0.0) / n)
    out = {"area_m2": area, "mean": [s / m for s in S], "fractiles": fr, "sum": S, "sum_sq": Q,
           "slope": slope, "intercept": icpt, "r_squared": r_sq, "rmse": rmse}
    if nn is not None:
        out["nn2_min"] = int(nn.min())
    return out
