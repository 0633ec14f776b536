"""Batches of independent clouds through pdd_decimate_batch, each cloud's
result against the oracle run on that cloud alone (bit for bit: kept,
removal order, removal costs), plus a single-cloud batch against
pdd_decimate."""
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


def _run_batch(ctx, clouds, keeps, k, **kw):
    import torch
    from paper_2311_17604_amd import pdd
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    x = torch.from_numpy(np.ascontiguousarray(np.concatenate(clouds), dtype=np.int32)).cuda()
    kept, order, oc = pdd.decimate_batch(ctx, x, off, keeps, k, **kw)
    ctx.stream.synchronize()
    return off, kept.cpu().numpy(), order.cpu().numpy(), oc.cpu().numpy().view(np.uint64)


def _check_against_oracle(oracle_mod, clouds, keeps, k, got):
    off, kept, order, oc = got
    ko = np.concatenate([[0], np.cumsum(keeps)])
    ro = np.concatenate([[0], np.cumsum([len(c) - kk for c, kk in zip(clouds, keeps)])])
    for s, (P, kk) in enumerate(zip(clouds, keeps)):
        ref = oracle_mod.decimate(P, k, int(kk), b=6)
        assert np.array_equal(kept[ko[s]:ko[s + 1]], ref[0]), ("kept", s)
        assert np.array_equal(order[ro[s]:ro[s + 1]], ref[1]), ("order", s)
        assert np.array_equal(oc[ro[s]:ro[s + 1]], ref[2]), ("order_cost", s)


@pytest.mark.parametrize("seed,k,frac", [(1, 8, 0.0), (2, 4, 0.05), (3, 16, 0.01), (4, 8, 0.3)])
def test_batch_random_clouds(gpu, oracle_mod, seed, k, frac):
    rng = np.random.default_rng(seed)
    clouds, keeps = [], []
    for s in range(30):
        n = int(rng.integers(k + 2, 1500))
        box = int(rng.choice([3, 20, 300, 5000]))
        clouds.append(scangen.random_cloud(n, box, int(rng.integers(0, 1 << 30))))
        keeps.append(int(rng.integers(1, n + 1)))
    got = _run_batch(gpu, clouds, keeps, k, round_frac=frac, check=True)
    _check_against_oracle(oracle_mod, clouds, keeps, k, got)


@pytest.mark.parametrize("frac", [0.01, 0.3])
def test_batch_round_graphs_equal_eager(gpu, oracle_mod, frac):
    # a batch's round is captured as two graphs around the budget cut (whose
    # sort runs eagerly between them); the same batch launched kernel by
    # kernel, and the oracle, agree, on one context with eager work between
    rng = np.random.default_rng(11)
    clouds, keeps = [], []
    for s in range(24):
        n = int(rng.integers(200, 3000))
        clouds.append(scangen.random_cloud(n, int(rng.choice([20, 300, 5000])), int(rng.integers(0, 1 << 30))))
        keeps.append(int(rng.integers(1, n // 2)))
    for eager in (False, True, False):
        got = _run_batch(gpu, clouds, keeps, 8, round_frac=frac, eager=eager)
        st = gpu.stats()
        _check_against_oracle(oracle_mod, clouds, keeps, 8, got)
        if eager:
            assert st["graph_rounds"] == 0
        else:
            assert 0 < st["graph_rounds"] <= st["rounds"], st


def test_batch_scans_uneven(gpu, oracle_mod):
    # scans of very different sizes and densities, keep ratios 10-50%
    clouds, keeps = [], []
    for s in range(12):
        P, keep = scangen.batch_scan(10000 + s, size_scale=0.02)
        clouds.append(P)
        keeps.append(keep)
    got = _run_batch(gpu, clouds, keeps, 8)
    _check_against_oracle(oracle_mod, clouds, keeps, 8, got)


def test_batch_of_one_equals_single(gpu, oracle_mod):
    import torch
    from paper_2311_17604_amd import pdd
    w = scangen.config(1, scale=0.2)
    got = _run_batch(gpu, [w.xyz], [w.keep], w.k)
    single = pdd.decimate(gpu, torch.from_numpy(w.xyz).cuda(), w.keep, w.k)
    gpu.stream.synchronize()
    assert np.array_equal(got[1], single[0].cpu().numpy())
    assert np.array_equal(got[2], single[1].cpu().numpy())
    assert np.array_equal(got[3], single[2].cpu().numpy().view(np.uint64))


def test_batch_identical_groups_and_tiny(gpu, oracle_mod):
    rng = np.random.default_rng(9)
    clouds, keeps = [], []
    for s in range(10):
        P = scangen.random_cloud(int(rng.integers(50, 800)), 2000, 100 + s)
        grp = np.repeat(P[:1], int(rng.integers(20, 200)), axis=0)
        Q = np.concatenate([P, grp])[rng.permutation(len(P) + len(grp))]
        clouds.append(np.ascontiguousarray(Q))
        keeps.append(int(rng.integers(1, len(Q) // 2)))
    clouds.append(np.array([[0, 0, 0], [5, 0, 0]], np.int32))   # two points
    keeps.append(1)
    got = _run_batch(gpu, clouds, keeps, 8)
    _check_against_oracle(oracle_mod, clouds, keeps, 8, got)


def test_batch_budget_cut_repeated(gpu, oracle_mod):
    # rounds whose A holds more than some clouds' remaining budget go
    # through the per-cloud budget cut (a segmented sort and compaction of
    # A); a large round share makes that happen in most rounds.  Repeated
    # on one context: the compacted A's length once came from a counter that
    # one block of the copy kernel could clear before another had read it.
    rng = np.random.default_rng(11)
    clouds, keeps = [], []
    for s in range(40):
        n = int(rng.integers(30, 900))
        clouds.append(scangen.random_cloud(n, int(rng.choice([3, 50, 2000])), int(rng.integers(0, 1 << 30))))
        keeps.append(int(rng.integers(1, max(2, n // 8))))
    for _ in range(4):
        got = _run_batch(gpu, clouds, keeps, 4, round_frac=0.3, check=True)
        _check_against_oracle(oracle_mod, clouds, keeps, 4, got)
