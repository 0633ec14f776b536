"""The quality measures (pdd_quality_measure) against the oracle
(oracle/quality_oracle.py) through the C ABI: per-point neighbour counts and
nearest distances element by element, the per-radius sums and fractiles
exactly, the regression figures to rounding."""
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


def _check(gpu, P, r2):
    import torch
    from oracle import quality_oracle as qo
    from paper_2311_17604_amd import pdd
    x = torch.from_numpy(np.ascontiguousarray(P, dtype=np.int32)).cuda()
    s, counts, nn2 = pdd.quality(gpu, x, r2)
    gpu.stream.synchronize()
    P3 = np.ascontiguousarray(P[:, :3])
    rc = qo.neighbor_counts(P3, r2)
    rn = qo.nn2(P3)
    assert np.array_equal(counts.cpu().numpy().astype(np.uint32), rc), "counts"
    assert np.array_equal(nn2.cpu().numpy(), rn), "nearest distances"
    ref = qo.summary(rc, r2, rn)
    assert s["m"] == len(P)
    assert s["sum"] == ref["sum"] and s["sum_sq"] == ref["sum_sq"]
    # fractiles come from per-radius count histograms of 4096 bins: a count
    # of 4095 or more reads as 4095, and the summary says so
    capped = any(v >= 4095 for row in ref["fractiles"] for v in row)
    assert s["fractile_capped"] == capped
    assert s["fractiles"] == [[min(v, 4095) for v in row] for row in ref["fractiles"]]
    assert s["nn2_min"] == ref["nn2_min"]
    for key in ("slope", "intercept", "r_squared", "rmse"):
        assert s[key] == pytest.approx(ref[key], rel=1e-9, abs=1e-9), key
    assert s["mean"] == pytest.approx(ref["mean"], rel=1e-12)
    return s


@pytest.mark.parametrize("n,box,seed", [(2000, 4, 1), (5000, 60, 2), (8000, 5000, 3), (2, 10, 4), (700, 1, 5)])
def test_random_clouds(gpu, n, box, seed):
    P = scangen.random_cloud(n, box, seed)
    _check(gpu, P, [0, 1, 4, 100, 2500, 40000])


def test_scan_and_its_decimation(gpu):
    import torch
    from paper_2311_17604_amd import pdd
    w = scangen.config(1, scale=0.1)
    r2 = [v * v for v in (20, 40, 80, 160, 320)]
    full = _check(gpu, w.xyz, r2)
    kept, _, _ = pdd.decimate(gpu, torch.from_numpy(w.xyz).cuda(), w.keep, w.k)
    gpu.stream.synchronize()
    K = w.xyz[np.sort(kept.cpu().numpy())]
    dec = _check(gpu, K, r2)
    # the decimated cloud is sparser and more even than the scan: its
    # nearest distances are never below the scan's smallest one
    assert dec["nn2_min"] >= full["nn2_min"]
    # and a 16-byte point stride gives the same
    K16 = np.concatenate([K, np.zeros((len(K), 1), np.int32)], axis=1)
    s16 = _check(gpu, K16, r2)
    assert s16["sum"] == dec["sum"]


def test_argument_errors(gpu):
    import torch
    from paper_2311_17604_amd import pdd
    x = torch.from_numpy(scangen.random_cloud(50, 100, 9)).cuda()
    for bad in ([100, 100], [100, 50], []):
        with pytest.raises(pdd.PddError) as e:
            pdd.quality(gpu, x, bad)
        assert e.value.status == pdd.PDD_EINVAL
    with pytest.raises(pdd.PddError):
        pdd.quality(gpu, x[:1], [100])


def test_decimation_is_more_even_than_a_random_subset(gpu):
    # the claim of Sec. 6 on one scan: the greedy keeps a set whose smallest
    # nearest-neighbour distance (Eq. 2) is larger, and whose neighbour
    # counts vary less, than a random subset of the same size
    import torch
    from paper_2311_17604_amd import pdd
    w = scangen.config(1, scale=0.25)
    x = torch.from_numpy(w.xyz).cuda()
    kept, _, _ = pdd.decimate(gpu, x, w.keep, w.k)
    gpu.stream.synchronize()
    rng = np.random.default_rng(3)
    rand = np.sort(rng.choice(len(w.xyz), w.keep, replace=False))
    r2 = [v * v for v in (50, 100, 150, 200)]
    sd, _, _ = pdd.quality(gpu, torch.from_numpy(w.xyz[np.sort(kept.cpu().numpy())]).cuda(), r2, with_counts=False)
    sr, _, _ = pdd.quality(gpu, torch.from_numpy(w.xyz[rand]).cuda(), r2, with_counts=False)
    assert sd["nn2_min"] > sr["nn2_min"]
    for r in range(len(r2)):
        band_d = sd["fractiles"][r][5] - sd["fractiles"][r][1]
        band_r = sr["fractiles"][r][5] - sr["fractiles"][r][1]
        assert band_d <= band_r, (r, sd["fractiles"][r], sr["fractiles"][r])
