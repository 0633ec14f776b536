"""HIP path against the oracle, element by element, through the C ABI."""
import numpy as np
import pytest

from paper_2311_17604_amd import scangen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2311_17604_amd import pdd
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = pdd.Context(0)
    yield ctx
    ctx.close()


def _dev(P):
    import torch
    return torch.from_numpy(np.ascontiguousarray(P, dtype=np.int32)).cuda()


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def gpu_knn(ctx, P, k, b, voxel=0):
    from paper_2311_17604_amd import pdd
    nbr, r2k, cost = pdd.knn_cost(ctx, _dev(P), k, b, voxel)
    return nbr.cpu().numpy(), r2k.cpu().numpy(), _u64(cost)


def gpu_decimate(ctx, P, keep, k, **kw):
    from paper_2311_17604_amd import pdd
    kept, order, oc = pdd.decimate(ctx, _dev(P), keep, k, **kw)
    ctx.stream.synchronize()
    return kept.cpu().numpy(), order.cpu().numpy(), _u64(oc)


def assert_knn_equal(P, k, b, got, ref):
    gn, gr, gc = got
    rn, rr, rc = ref
    assert np.array_equal(gc, rc), "cost"
    assert np.array_equal(gr, rr), "r2k"
    Pi = P.astype(np.int64)
    K = k + b
    rows = np.arange(len(P))[:, None]
    valid = rn >= 0
    assert np.array_equal(gn >= 0, valid)
    gd = np.where(valid, ((Pi[np.maximum(gn, 0)] - Pi[rows]) ** 2).sum(-1), -1)
    rd = np.where(valid, ((Pi[np.maximum(rn, 0)] - Pi[rows]) ** 2).sum(-1), -1)
    assert np.array_equal(gd, rd), "neighbour distances"
    # below each row's last distance the set of points at every distance is
    # unique (order among equal distances is unspecified); at the last
    # distance any point at that distance is valid (gd == rd, no self, no repeat)
    last = rd.max(axis=1, keepdims=True)
    strict = valid & (rd < last)
    big = np.iinfo(np.int64).max
    gkey = np.where(strict, gd, big)
    rkey = np.where(strict, rd, big)
    go = np.lexsort((np.where(strict, gn, big), gkey), axis=1)
    ro = np.lexsort((np.where(strict, rn, big), rkey), axis=1)
    gs = np.take_along_axis(np.where(strict, gn, -1), go, axis=1)
    rs = np.take_along_axis(np.where(strict, rn, -1), ro, axis=1)
    assert np.array_equal(gs, rs), "neighbour ids"
    assert not (gn == rows).any()
    for i in np.flatnonzero((valid & (rd == last)).any(axis=1))[:2000]:
        v = gn[i][gn[i] >= 0]
        assert len(set(v.tolist())) == len(v)


KNN_CASES = [(300, 5, 8, 0, 0, 1), (2000, 40, 8, 8, 0, 2), (3000, 3000, 16, 8, 0, 3), (500, 2, 4, 4, 3, 4),
             (40, 1000, 30, 2, 2, 5), (5000, 100000, 8, 6, 12, 6), (9, 10, 8, 8, 0, 7)]


@pytest.mark.parametrize("n,box,k,b,voxel,seed", KNN_CASES)
def test_knn_cost_random(gpu, oracle_mod, n, box, k, b, voxel, seed):
    P = scangen.random_cloud(n, box, seed)
    got = gpu_knn(gpu, P, k, b, voxel)
    ref = oracle_mod.knn_cost(P, k, b)
    assert_knn_equal(P, k, b, got, ref)


@pytest.mark.parametrize("k,b", [(8, 8), (16, 0)])
def test_knn_cost_scan(gpu, oracle_mod, k, b):
    P = scangen.config(1).xyz
    got = gpu_knn(gpu, P, k, b)
    ref = oracle_mod.knn_cost(P, k, b)
    assert_knn_equal(P, k, b, got, ref)


def _dec_cases():
    rng = np.random.default_rng(17)
    out = []
    for t in range(40):
        k = int(rng.choice([1, 2, 3, 4, 6, 8, 16]))
        n = int(rng.integers(k + 2, 400))
        box = int(rng.choice([2, 5, 20, 200, 5000]))
        keep = int(rng.integers(1, n + 1))
        frac = float(rng.choice([0.01, 0.05, 0.3, 1.0]))
        voxel = int(rng.choice([0, 2, 4, 8]))
        b = int(rng.choice([0, 2, 8]))
        out.append((n, box, k, b, keep, frac, voxel, int(rng.integers(0, 1 << 30))))
    return out


@pytest.mark.parametrize("n,box,k,b,keep,frac,voxel,seed", _dec_cases())
def test_decimate_random(gpu, oracle_mod, n, box, k, b, keep, frac, voxel, seed):
    P = scangen.random_cloud(n, box, seed)
    ref = oracle_mod.decimate(P, k, keep, b=2)
    got = gpu_decimate(gpu, P, keep, k, b=b, round_frac=frac, voxel_log2=voxel, check=True)
    assert np.array_equal(got[0], ref[0]), "kept"
    assert np.array_equal(got[1], ref[1]), "order"
    assert np.array_equal(got[2], ref[2]), "order_cost"


@pytest.mark.parametrize("n", [63, 64, 65, 128, 4096, 4097])
@pytest.mark.parametrize("box,frac", [(20, 0.3), (200, 0.01)])
def test_decimate_word_boundaries(gpu, oracle_mod, n, box, frac):
    # the survivors of a round are ranked through one bit per point in 64-bit
    # words: clouds that end on, just before and just after a word boundary
    P = scangen.random_cloud(n, box, n + box)
    keep = max(1, n // 4)
    ref = oracle_mod.decimate(P, 8, keep, b=2)
    got = gpu_decimate(gpu, P, keep, 8, round_frac=frac, check=True)
    for g, r, name in zip(got, ref, ("kept", "order", "order_cost")):
        assert np.array_equal(g, r), name


@pytest.mark.parametrize("scale,frac", [(0.1, 0.03), (1.0, 0.03), (1.0, 0.1)])
def test_decimate_scan(gpu, oracle_mod, scale, frac):
    w = scangen.config(1, scale=scale)
    ref = oracle_mod.decimate(w.xyz, w.k, w.keep, b=6)
    got = gpu_decimate(gpu, w.xyz, w.keep, w.k, round_frac=frac)
    for g, r, name in zip(got, ref, ("kept", "order", "order_cost")):
        assert np.array_equal(g, r), name


@pytest.mark.parametrize("idx", [3, 5])
def test_decimate_merged_crop(gpu, oracle_mod, idx):
    # the crop of a merged multi-station cloud (uneven density: the ground
    # around one tripod plus the sparse hits of the other stations) on a
    # 1/100 ray grid, about 200k points
    w = scangen.config(idx, scale=0.01, crop=True)
    ref = oracle_mod.decimate(w.xyz, w.k, w.keep, b=6)
    got = gpu_decimate(gpu, w.xyz, w.keep, w.k)
    for g, r, name in zip(got, ref, ("kept", "order", "order_cost")):
        assert np.array_equal(g, r), name


def _dup_cloud(seed, n_base, box, sizes):
    """Random cloud plus groups of identical points (copies of random base
    points), shuffled so that each group's members interleave in index order."""
    rng = np.random.default_rng(seed)
    P = scangen.random_cloud(n_base, box, seed)
    groups = [np.repeat(P[rng.integers(0, n_base)][None, :], m, axis=0) for m in sizes]
    Q = np.concatenate([P] + groups)
    return np.ascontiguousarray(Q[rng.permutation(len(Q))])


@pytest.mark.parametrize("seed,k,keep_frac,frac", [(1, 8, 0.25, 0.01), (2, 16, 0.1, 0.01), (3, 8, 0.5, 0.3),
                                                   (4, 16, 0.2, 1.0), (5, 4, 0.05, 0.05)])
def test_decimate_identical_groups(gpu, oracle_mod, seed, k, keep_frac, frac):
    # large groups of identical points: all members share one cost, and a
    # member with k identical points ranked below it goes in the same round
    P = _dup_cloud(seed, 3000, 3000, [400, 250, 100, 40, 17, 16, 9, 5, 3, 2, 2])
    keep = max(1, int(len(P) * keep_frac))
    ref = oracle_mod.decimate(P, k, keep, b=8)
    got = gpu_decimate(gpu, P, keep, k, round_frac=frac, check=True)
    for g, r, name in zip(got, ref, ("kept", "order", "order_cost")):
        assert np.array_equal(g, r), name


def test_decimate_edges(gpu, oracle_mod):
    # keep everything, keep one, two points, all coincident, a line, 16-byte stride
    P = scangen.random_cloud(64, 50, 9)
    for keep in (64, 1, 63):
        ref = oracle_mod.decimate(P, 4, keep)
        got = gpu_decimate(gpu, P, keep, 4)
        assert all(np.array_equal(g, r) for g, r in zip(got, ref)), keep
    P2 = np.array([[0, 0, 0], [3, 4, 0]], np.int32)
    assert all(np.array_equal(g, r) for g, r in zip(gpu_decimate(gpu, P2, 1, 1), oracle_mod.decimate(P2, 1, 1)))
    P3 = np.zeros((50, 3), np.int32) + 7
    assert all(np.array_equal(g, r) for g, r in zip(gpu_decimate(gpu, P3, 10, 8), oracle_mod.decimate(P3, 8, 10)))
    P4 = np.zeros((300, 3), np.int32)
    P4[:, 0] = np.arange(300)
    assert all(np.array_equal(g, r) for g, r in zip(gpu_decimate(gpu, P4, 30, 1), oracle_mod.decimate(P4, 1, 30)))
    P5 = scangen.config(1, scale=0.02).xyz
    P16 = np.concatenate([P5, np.full((len(P5), 1), 0x00AABBCC, np.int32)], axis=1)
    ref = oracle_mod.decimate(P5, 8, len(P5) // 4)
    got = gpu_decimate(gpu, P16, len(P5) // 4, 8)
    assert all(np.array_equal(g, r) for g, r in zip(got, ref))


def test_decimate_range_error(gpu):
    from paper_2311_17604_amd import pdd
    P = np.array([[0, 0, 0], [1 << 21, 0, 0], [5, 5, 5]], np.int32)
    with pytest.raises(pdd.PddError) as e:
        gpu_decimate(gpu, P, 2, 1)
    assert e.value.status == pdd.PDD_ERANGE


@pytest.mark.parametrize("scale,frac", [(0.3, 0.01), (0.3, 0.3)])
def test_round_graph_equals_eager(gpu, oracle_mod, scale, frac):
    # a single cloud's round is captured once as a hipGraph and replayed
    # every round (re-captured after the rebuilds between rounds); the same
    # decimation with every kernel launched eagerly, and the oracle, agree,
    # on one context with eager work between the graph runs
    w = scangen.config(1, scale=scale)
    ref = oracle_mod.decimate(w.xyz, w.k, w.keep, b=6)
    for eager in (False, True, False):
        got = gpu_decimate(gpu, w.xyz, w.keep, w.k, round_frac=frac, eager=eager)
        st = gpu.stats()
        for g, r, name in zip(got, ref, ("kept", "order", "order_cost")):
            assert np.array_equal(g, r), (name, eager)
        if eager:
            assert st["graph_rounds"] == 0
        else:
            assert 0 < st["graph_rounds"] <= st["rounds"], st
