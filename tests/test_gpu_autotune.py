"""The autotuner through the C ABI: the settings it returns are in range,
and a decimation with them gives the same result as with the defaults and
as the oracle (the settings change only the time)."""
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


def test_autotune_settings_keep_result(gpu, oracle_mod):
    import torch
    from paper_2311_17604_amd import pdd
    w = scangen.config(1, scale=0.3)
    x = torch.from_numpy(w.xyz).cuda()
    t = pdd.autotune(gpu, x, w.keep, w.k, sample=20000)
    assert t["b"] in (0, 4, 12, 16) and 0 < t["round_frac"] <= 0.04
    assert t["voxel_log2"] == 0 or 2 <= t["voxel_log2"] <= 20
    assert t["best_ms"] > 0
    tuned = pdd.decimate(gpu, x, w.keep, w.k, b=t["b"], voxel_log2=t["voxel_log2"], round_frac=t["round_frac"])
    plain = pdd.decimate(gpu, x, w.keep, w.k)
    gpu.stream.synchronize()
    ref = oracle_mod.decimate(w.xyz, w.k, w.keep, b=6)
    for a_, b_, r_, name in zip(tuned, plain, ref, ("kept", "order", "order_cost")):
        a_, b_ = a_.cpu().numpy(), b_.cpu().numpy()
        if name == "order_cost":
            a_, b_ = a_.view(np.uint64), b_.view(np.uint64)
        assert np.array_equal(a_, b_) and np.array_equal(a_, r_), name


def test_autotune_batch_settings_keep_result(gpu, oracle_mod):
    # 24 scans of the batch generator at 1/400 size; the tuner samples every
    # few scans, and the batch decimated with its choice equals the oracle
    # run on each scan alone
    import torch
    from paper_2311_17604_amd import pdd
    w = scangen.batch_config(24, scale=1 / 400, base_seed=10000)
    x = torch.from_numpy(w.xyz).cuda()
    t = pdd.autotune_batch(gpu, x, w.offsets, w.keeps, w.k, sample=20000)
    assert t["b"] in (0, 4, 16, 24) and 0 < t["round_frac"] <= 0.02
    assert t["voxel_log2"] == 0 and t["best_ms"] > 0
    kept, order, oc = pdd.decimate_batch(gpu, x, w.offsets, w.keeps, w.k, b=t["b"], round_frac=t["round_frac"])
    gpu.stream.synchronize()
    kept, order, oc = kept.cpu().numpy(), order.cpu().numpy(), oc.cpu().numpy().view(np.uint64)
    ko = np.concatenate([[0], np.cumsum(w.keeps)])
    sizes = np.diff(w.offsets)
    ro = np.concatenate([[0], np.cumsum(sizes - w.keeps)])
    for s in range(len(w.keeps)):
        P = w.xyz[w.offsets[s]:w.offsets[s + 1]]
        ref = oracle_mod.decimate(P, w.k, int(w.keeps[s]), b=6)
        assert np.array_equal(kept[ko[s]:ko[s + 1]], ref[0]), ("kept", s)
        assert np.array_equal(order[ro[s]:ro[s + 1]], ref[1]), ("order", s)
        assert np.array_equal(oc[ro[s]:ro[s + 1]], ref[2]), ("order_cost", s)
