"""Pins of the CPU oracle against things other than itself.

* k-NN lists: O(n^2) brute force with an explicit (d2, index) sort, and
  scipy's cKDTree (a library routine) on the d2 multisets.
* The fixed-point cost: the floor definition and its error against the
  exact rational value of Eq. 12 (Sec. 4.2), computed with Fractions.
* The greedy: a brute-force greedy that recomputes every cost from scratch
  before each removal (Sec. 4: remove the highest-cost sample, costs of the
  rest updated), on tiny inputs full of duplicates and ties.
* Hand-derived cases: 1 mm line, alternating pair spacing, a duplicate
  pair, the two-close-points case of Fig. 3, k = 1 ranking = ascending
  nearest-neighbour distance (Eq. 11).
* Invariants (Sec. 5, step 2 and Sec. 3): costs never rise, removal keys
  strictly decrease, exactly keep points remain, results independent of b.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2311_17604_amd import scangen

TWO56 = 1 << 56


def brute_knn(P, K):
    P = P.astype(np.int64)
    n = len(P)
    D = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    nbr = np.full((n, K), -1, dtype=np.int64)
    d2 = np.full((n, K), -1, dtype=np.int64)
    idx = np.arange(n)
    for i in range(n):
        m = idx != i
        cand, dd = idx[m], D[i][m]
        o = np.lexsort((cand, dd))[:K]
        nbr[i, :len(o)] = cand[o]
        d2[i, :len(o)] = dd[o]
    return nbr, d2


def brute_greedy(P, k, keep):
    """Recompute every cost from its definition before each removal."""
    P = [tuple(int(c) for c in p) for p in P]
    n = len(P)
    D = [[sum((a - b) ** 2 for a, b in zip(P[i], P[j])) for j in range(n)] for i in range(n)]

    def t(d):
        return 1 << 58 if d == 0 else TWO56 // d

    alive = set(range(n))
    order, costs = [], []
    while len(alive) > keep:
        best = None
        for i in sorted(alive):
            ds = sorted(D[i][j] for j in alive if j != i)[:k]
            w = sum(t(d) for d in ds)
            if best is None or w > best[0]:
                best = (w, i)
        order.append(best[1])
        costs.append(best[0])
        alive.remove(best[1])
    return sorted(alive), order, costs


# --------------------------------------------------------------------------
# k-NN
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,box,K,seed", [(300, 5, 8, 1), (800, 40, 16, 2), (1500, 2000, 24, 3),
                                          (50, 2, 32, 4), (9, 1000, 8, 5)])
def test_knn_matches_bruteforce(oracle_mod, n, box, K, seed):
    P = scangen.random_cloud(n, box, seed)
    nbr, d2 = oracle_mod.knn(P, K)
    bn, bd = brute_knn(P, K)
    assert np.array_equal(d2, bd)
    assert np.array_equal(nbr, bn)


def test_knn_matches_ckdtree_on_scan(oracle_mod):
    from scipy.spatial import cKDTree
    P = scangen.config(1, scale=0.25).xyz
    K = 12
    nbr, d2 = oracle_mod.knn(P, K)
    dist, _ = cKDTree(P.astype(np.float64)).query(P.astype(np.float64), k=K + 1)
    ref = np.rint(dist[:, 1:] ** 2).astype(np.int64)
    # the point itself is at distance 0 but so is any duplicate: compare the
    # multiset of the K+1 smallest including one zero for the point itself
    full = np.rint(dist ** 2).astype(np.int64)
    mine = np.concatenate([np.zeros((len(P), 1), np.int64), d2], axis=1)
    assert np.array_equal(np.sort(full, axis=1), np.sort(mine, axis=1))
    assert ref.shape == d2.shape
    # neighbours are at the distances reported
    Pi = P.astype(np.int64)
    rows = np.arange(len(P))[:, None]
    assert np.array_equal(((Pi[nbr] - Pi[rows]) ** 2).sum(-1), d2)


# --------------------------------------------------------------------------
# the cost term and Eq. 12
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d2", [1, 2, 3, 5, 7, 1000, 999_983, 2**20 + 1, 3 * 2**42 - 1, 2**44 + 12345])
def test_term_is_floor_of_2_56_over_d2(oracle_mod, d2):
    t = oracle_mod.term(d2)
    assert t * d2 <= TWO56 < (t + 1) * d2


def test_term_zero_distance_ranks_above_every_finite_term(oracle_mod):
    assert oracle_mod.term(0) == 1 << 58
    assert oracle_mod.term(0) > oracle_mod.term(1) == TWO56
    # k <= 32 duplicates still fit a uint64 cost
    assert 32 * oracle_mod.term(0) <= 2**64 - 1


@pytest.mark.parametrize("k,seed,box", [(1, 11, 300), (3, 12, 300), (6, 13, 60), (8, 14, 5000)])
def test_cost_is_fixed_point_of_eq11(oracle_mod, k, seed, box):
    """W = sum over the k nearest of 1/d^2 (Eq. 12), scaled by 2^56, each
    term floored: 0 <= 2^56 W_exact - W < k for clouds without duplicates."""
    P = scangen.random_cloud(200, box, seed)
    P = np.unique(P, axis=0)
    nbr, r2k, cost = oracle_mod.knn_cost(P, k, 0)
    Pi = P.astype(np.int64)
    n = len(P)
    for i in range(n):
        d = sorted(int(((Pi[i] - Pi[j]) ** 2).sum()) for j in range(n) if j != i)[:k]
        exact = sum(Fraction(1, x) for x in d) * TWO56
        err = exact - int(cost[i])
        assert 0 <= err < k, (i, err)
        assert r2k[i] == d[-1]


def test_k1_ranking_is_ascending_nearest_distance(oracle_mod):
    """Eq. 11: with k = 1 the cost is 1/d_p^2, so ranking by cost (desc,
    then index) is ranking by nearest distance (asc, then index)."""
    P = scangen.config(1, scale=0.05).xyz
    _, r2k, cost = oracle_mod.knn_cost(P, 1, 0)
    idx = range(len(P))
    by_cost = sorted(idx, key=lambda i: (-int(cost[i]), i))
    by_dist = sorted(idx, key=lambda i: (int(r2k[i]), i))
    assert by_cost == by_dist


# --------------------------------------------------------------------------
# the greedy
# --------------------------------------------------------------------------

def _cases():
    out = []
    rng = np.random.default_rng(7)
    for k in (1, 2, 3, 4, 6, 8):
        for box in (3, 10, 60):
            n = int(rng.integers(12, 40))
            keep = int(rng.integers(1, n))
            out.append((k, box, n, keep, int(rng.integers(0, 1 << 30))))
    return out


@pytest.mark.parametrize("k,box,n,keep,seed", _cases())
def test_greedy_matches_bruteforce(oracle_mod, k, box, n, keep, seed):
    P = scangen.random_cloud(n, box, seed)
    kept, order, oc = oracle_mod.decimate(P, k, keep, b=2, check=True)
    bk, bo, bc = brute_greedy(P, k, keep)
    assert list(kept) == bk
    assert list(order) == bo
    assert [int(c) for c in oc] == bc


def test_greedy_matches_bruteforce_lidar_crop(oracle_mod):
    P = scangen.config(1, scale=0.25).xyz
    # a small spatial crop with the polar cluster: every point near the top
    top = np.argsort(-P[:, 2].astype(np.int64))[:120]
    Q = P[np.sort(top)]
    for k in (1, 4, 8):
        kept, order, oc = oracle_mod.decimate(Q, k, 30, b=3, check=True)
        bk, bo, bc = brute_greedy(Q, k, 30)
        assert list(kept) == bk and list(order) == bo and [int(c) for c in oc] == bc


def test_line_1mm_k1_removes_in_index_order(oracle_mod):
    n = 50
    P = np.zeros((n, 3), np.int32)
    P[:, 0] = np.arange(n)
    kept, order, oc = oracle_mod.decimate(P, 1, 5, b=0, check=True)
    assert list(order) == list(range(45))
    assert list(kept) == list(range(45, 50))
    assert all(int(c) == TWO56 for c in oc)


def test_alternating_pairs_keep_second_members(oracle_mod):
    """Gaps 1, 2, 1, 2, ...: each pair's first member goes, left to right."""
    n = 40
    x = np.cumsum([0] + [1 if i % 2 == 0 else 2 for i in range(n - 1)])
    P = np.zeros((n, 3), np.int32)
    P[:, 0] = x
    kept, order, oc = oracle_mod.decimate(P, 1, n // 2, b=2, check=True)
    assert list(kept) == list(range(1, n, 2))
    assert list(order) == list(range(0, n, 2))


def test_duplicate_pair_lower_index_first_with_2_58(oracle_mod):
    P = np.array([[0, 0, 0], [5000, 0, 0], [0, 5000, 0], [777, 777, 7], [777, 777, 7], [0, 0, 5000]],
                 np.int32)
    for k in (1, 2, 4):
        kept, order, oc = oracle_mod.decimate(P, k, 5, b=1, check=True)
        assert list(order) == [3]
        assert int(oc[0]) >= 1 << 58
        assert list(kept) == [0, 1, 2, 4, 5]


def test_fig3_two_close_points(oracle_mod):
    """Fig. 3: three spread points and two close ones at equal nearest
    distance.  k = 1 ties them (the lower index goes); k = 4 removes the
    one nearer the spread points (the 'blue' one)."""
    black = [[0, 0, 0], [1000, 0, 0], [500, 866, 0]]
    orange = [500, 289, 0]      # near the triangle's centre
    blue = [500, 189, 0]        # 100 mm away, towards the edge 0-1
    P = np.array(black + [orange, blue], np.int32)
    _, o1, c1 = oracle_mod.decimate(P, 1, 4, b=0, check=True)
    assert list(o1) == [3]
    _, o4, c4 = oracle_mod.decimate(P, 4, 4, b=0, check=True)
    assert list(o4) == [4]
    # exact rational Eq. 12 agrees on which of the two is denser
    Q = P.tolist()

    def w(i):
        return sum(Fraction(1, sum((a - b) ** 2 for a, b in zip(Q[i], Q[j]))) for j in range(5) if j != i)
    assert w(4) > w(3)


@pytest.mark.parametrize("k,b", [(8, 0), (8, 6), (8, 24), (16, 8)])
def test_result_independent_of_buffer_and_invariants(oracle_mod, k, b):
    P = scangen.config(1, scale=0.1).xyz
    keep = len(P) // 10
    ref = oracle_mod.decimate(P, k, keep, b=0, check=True)
    got = oracle_mod.decimate(P, k, keep, b=b, check=True)
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)
    kept, order, oc = got
    assert len(kept) == keep and len(set(kept) | set(order)) == len(P)
    assert np.all(np.diff(kept) > 0)
