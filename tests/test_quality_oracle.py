"""Pins of the quality-measure oracle (oracle/quality_oracle.py): counts and
nearest distances against brute force, counts on a lattice against the
lattice-point count of a disc, fractiles against numpy's 'lower' quantile,
and the regression against scipy's linregress over the explicit pairs."""
import math

import numpy as np
import pytest

from oracle import quality_oracle as qo
from paper_2311_17604_amd import scangen


def _brute_counts(P, r2):
    P = P.astype(np.int64)
    d2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.iinfo(np.int64).max)
    return np.stack([(d2 <= v).sum(1) for v in r2], axis=1).astype(np.uint32), d2.min(1)


@pytest.mark.parametrize("n,box,seed", [(300, 4, 1), (500, 60, 2), (400, 5000, 3), (2, 10, 4)])
def test_counts_and_nn_match_brute_force(n, box, seed):
    P = scangen.random_cloud(n, box, seed)
    r2 = [0, 1, 9, 100, 2500, 10**6]
    bc, bn = _brute_counts(P, r2)
    assert np.array_equal(qo.neighbor_counts(P, r2), bc)
    assert np.array_equal(qo.nn2(P), bn)


def test_lattice_counts_are_disc_lattice_counts():
    # a 41 x 41 square lattice at 7 mm in a plane: a point at least r from
    # the border has as many neighbours within r as the disc of radius r/7
    # holds lattice points, less itself
    s, N = 7, 41
    ij = np.stack(np.meshgrid(np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 2)
    P = np.concatenate([ij * s, np.zeros((len(ij), 1), np.int64)], axis=1).astype(np.int32)
    r2 = [49, 98, 196, 441, 1225]
    c = qo.neighbor_counts(P, r2)
    for r, v in enumerate(r2):
        rr = v / (s * s)
        k = int(math.floor(math.sqrt(rr)))
        disc = sum(1 for a in range(-k, k + 1) for b in range(-k, k + 1) if a * a + b * b <= rr) - 1
        margin = int(math.ceil(math.sqrt(rr)))
        inner = (ij[:, 0] >= margin) & (ij[:, 0] < N - margin) & (ij[:, 1] >= margin) & (ij[:, 1] < N - margin)
        assert np.all(c[inner, r] == disc), (v, disc)


def test_fractiles_and_regression():
    rng = np.random.default_rng(5)
    counts = rng.integers(0, 50, size=(997, 4)).astype(np.uint32)
    counts[:, 1] += 20
    counts[:, 2] += 45
    counts[:, 3] += 80
    r2 = [10**6, 4 * 10**6, 9 * 10**6, 16 * 10**6]
    s = qo.summary(counts, r2)
    for r in range(4):
        want = [int(np.quantile(counts[:, r], q, method="lower")) for q in qo.FRACTILES]
        assert s["fractiles"][r] == want
        assert s["mean"][r] == pytest.approx(counts[:, r].mean(), rel=1e-12)
    from scipy import stats
    x = np.repeat(np.array([[math.pi * v / 1e6 for v in r2]]), len(counts), axis=0).ravel()
    y = counts.astype(np.float64).ravel()
    lr = stats.linregress(x, y)
    assert s["slope"] == pytest.approx(lr.slope, rel=1e-9)
    assert s["intercept"] == pytest.approx(lr.intercept, rel=1e-9, abs=1e-9)
    assert s["r_squared"] == pytest.approx(lr.rvalue ** 2, rel=1e-9)
    res = y - (lr.intercept + lr.slope * x)
    assert s["rmse"] == pytest.approx(math.sqrt((res ** 2).mean()), rel=1e-7)


def test_uniform_surface_density_is_the_slope():
    # points on a plane at a known density: the slope of count against area
    # (m^2) approaches that density (here 40000 points on 400 m^2: 100 per m^2)
    rng = np.random.default_rng(7)
    n = 40000
    P = np.concatenate([rng.integers(0, 20000, size=(n, 2)), np.zeros((n, 1), np.int64)], axis=1).astype(np.int32)
    r2 = [v * v for v in (100, 150, 200, 250, 300)]
    c = qo.neighbor_counts(P, r2)
    keep = (P[:, 0] > 400) & (P[:, 0] < 19600) & (P[:, 1] > 400) & (P[:, 1] < 19600)
    s = qo.summary(c[keep], r2)
    assert s["slope"] == pytest.approx(n / 400.0, rel=0.03)
    assert s["r_squared"] > 0.8
