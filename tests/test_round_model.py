"""The exact parallel round rule, as a small numpy model, against the oracle.

A round takes the m <= B highest keys A (B = removals still to do).  For x
in A let H(x) be the points of A above x, rho'(x) the k-th smallest d2 from
x to the alive points not in H(x) (x excluded), and rho(x | y) the k-th
smallest d2 from y to the alive points not in H(x) (x, y excluded).  x is
blocked if some y in H(x) has d2(x, y) < rho'(x) or d2(x, y) < rho(x | y);
every unblocked x is removed at once with its current cost.  Costs never
rise after a removal (Sec. 5, step 2), which makes the result equal to the
sequential greedy's (Sec. 4) for any m.  The GPU rounds implement this rule
(blocking more where their stored lists cannot decide).  The cases also keep
the weaker rule that measures both radii to L = alive minus A, and the two
counterexamples to a rule without such radii and without m <= B.
"""
import numpy as np
import pytest

from paper_2311_17604_amd import scangen

TWO56 = 1 << 56


def _d2(P):
    P = P.astype(np.int64)
    return ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)


def _costs(D, alive, k):
    idx = np.flatnonzero(alive)
    W = {}
    for i in idx:
        ds = np.sort(D[i, idx[idx != i]])[:k]
        W[int(i)] = sum((1 << 58) if d == 0 else TWO56 // int(d) for d in ds)
    return W


def _kth(D, i, pool, k):
    pool = [z for z in pool if z != i]
    return np.sort(D[i, pool])[k - 1] if len(pool) >= k else np.inf


def round_model(P, k, keep, frac, rule="stable"):
    n = len(P)
    D = _d2(P)
    alive = np.ones(n, bool)
    events = []
    rounds = 0
    while len(events) < n - keep:
        rounds += 1
        B = n - keep - len(events)
        W = _costs(D, alive, k)
        S = sorted(W, key=lambda i: (-W[i], i))
        m = min(B, max(1, int(np.ceil(frac * len(S)))))
        A, L = S[:m], S[m:]
        rank = {x: r for r, x in enumerate(S)}  # lower rank = higher key
        blocked = set()
        for x in A:
            H = S[:rank[x]]
            if rule == "stable":
                rest = S[rank[x]:]          # not above x (x itself dropped by _kth)
                rx = _kth(D, x, rest, k)
                for y in H:
                    if D[x, y] < rx or D[x, y] < _kth(D, y, [z for z in rest if z != x], k):
                        blocked.add(x)
                        break
            else:
                rx = _kth(D, x, L, k)
                for y in H:
                    if D[x, y] < rx or D[x, y] < _kth(D, y, L, k):
                        blocked.add(x)
                        break
        R = [x for x in A if x not in blocked]
        assert R, "the top key is never blocked"
        for x in R:
            events.append((W[x], x))
            alive[x] = False
    events.sort(key=lambda e: (-e[0], e[1]))
    return np.flatnonzero(alive), [e[1] for e in events], [e[0] for e in events], rounds


def literal_rule(P, k, keep):
    """Strict local maxima over kNN and reverse kNN removed at once, while
    they fit the budget; then exact order.  Not exact (kept as regression)."""
    n = len(P)
    D = _d2(P)
    alive = np.ones(n, bool)
    removed = []
    while len(removed) < n - keep:
        B = n - keep - len(removed)
        W = _costs(D, alive, k)
        idx = np.flatnonzero(alive)
        key = {i: (W[i], -i) for i in W}
        nb = {}
        for i in idx:
            o = idx[idx != i]
            nb[int(i)] = set(int(j) for j in o[np.lexsort((o, D[i, o]))[:k]])
        rev = {int(i): set() for i in idx}
        for i in nb:
            for j in nb[i]:
                rev[j].add(i)
        cand = [i for i in W if all(key[i] > key[j] for j in nb[i] | rev[i])]
        if len(cand) > B:
            top = max(W, key=lambda i: key[i])
            cand = [top]
        for i in cand:
            alive[i] = False
            removed.append(i)
    return np.flatnonzero(alive)


def _cases():
    rng = np.random.default_rng(2311)
    out = []
    for t in range(60):
        k = int(rng.choice([1, 2, 3, 4, 6, 8]))
        n = int(rng.integers(k + 2, 22))
        box = int(rng.choice([2, 4, 10, 40]))
        keep = int(rng.integers(1, n))
        frac = float(rng.choice([0.01, 0.1, 0.3, 0.5, 1.0]))
        out.append((k, n, box, keep, frac, int(rng.integers(0, 1 << 30))))
    return out


@pytest.mark.parametrize("k,n,box,keep,frac,seed", _cases())
@pytest.mark.parametrize("rule", ["stable", "outside_A"])
def test_round_rule_equals_sequential_greedy(oracle_mod, k, n, box, keep, frac, seed, rule):
    P = scangen.random_cloud(n, box, seed)
    kept, order, oc = oracle_mod.decimate(P, k, keep, b=2)
    mk, mo, mc, _ = round_model(P, k, keep, frac, rule)
    assert np.array_equal(kept, mk)
    assert list(order) == mo
    assert [int(c) for c in oc] == mc


def test_round_rule_on_scan_crop_takes_few_rounds(oracle_mod):
    P = scangen.config(1, scale=0.01).xyz[:300]
    kept, order, oc = oracle_mod.decimate(P, 8, 75, b=4)
    mk, mo, mc, rounds = round_model(P, 8, 75, 0.05)
    assert np.array_equal(kept, mk) and list(order) == mo
    assert rounds < 225 / 2


def test_stable_rule_needs_fewer_rounds_on_polar_cluster(oracle_mod):
    """Near-duplicate cluster of the top scan row: counting lower points of A
    as stable neighbours frees most of the cluster at once."""
    P = scangen.config(1, scale=0.25).xyz
    Q = P[np.sort(np.argsort(-P[:, 2].astype(np.int64))[:160])]
    kept, order, _ = oracle_mod.decimate(Q, 4, 40, b=2)
    a = round_model(Q, 4, 40, 0.3, "stable")
    b = round_model(Q, 4, 40, 0.3, "outside_A")
    assert np.array_equal(a[0], kept) and np.array_equal(b[0], kept) and a[1] == list(order)
    assert a[3] < b[3]


def test_counterexample_budget(oracle_mod):
    P = np.array([(0, 0, 1), (0, 0, 0), (2, 1, 0), (1, 1, 2), (0, 2, 0), (0, 1, 0)], np.int32)
    kept, order, _ = oracle_mod.decimate(P, 1, 4, b=0)
    assert list(order) == [0, 1]
    assert not np.array_equal(literal_rule(P, 1, 4), kept)
    assert np.array_equal(round_model(P, 1, 4, 1.0)[0], kept)


def test_counterexample_entering_neighbour(oracle_mod):
    P = np.array([(12, 21, 0), (24, 0, 1), (24, 12, 0), (26, 30, 1), (32, 36, 2), (29, 50, 1),
                  (27, 48, 0), (40, 9, 1), (0, 17, 2)], np.int32)
    kept, _, _ = oracle_mod.decimate(P, 3, 4, b=0)
    assert list(kept) == [1, 5, 7, 8]
    assert list(literal_rule(P, 3, 4)) == [3, 5, 7, 8]
    assert np.array_equal(round_model(P, 3, 4, 1.0)[0], kept)
