"""The learned search-radius bound through the C ABI: the network's forward
pass and gradient against the float64 reference (oracle/mlp_oracle.py) with
the same bfloat16 operand rounding, training on k-NN radii of generated
scans, and what the trained network gains on a held-out scan with the
results unchanged.

Tolerances: the GPU accumulates the bf16 products in fp32 and the reference
in float64, and both round the same operands to bf16.  A rounding boundary
can still fall between the two accumulations for an occasional hidden value
(one bf16 step, 2^-8 relative), so outputs agree to about 1e-3 of their
scale and gradients to about 1e-2 of their norm."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo
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


def _bits_to_f64(t):
    a = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32).astype(np.float64)


def _f64_to_bits(x):
    r = np.asarray(mo.bf16_round(x), dtype=np.float32).view(np.uint32) >> 16
    return r.astype(np.uint16).view(np.int16)


def _init(seed, y_mean=0.0):
    rng = np.random.default_rng(seed)
    return mo.pack({"W1": rng.normal(0, np.sqrt(2 / 64), (64, 64)), "b1": np.zeros(64),
                    "W2": rng.normal(0, np.sqrt(2 / 64), (64, 64)), "b2": np.zeros(64),
                    "w3": rng.normal(0, 0.05, 64), "b3": np.array([y_mean])}).astype(np.float32)


def _features(seed, n):
    rng = np.random.default_rng(seed)
    return np.log1p(rng.integers(0, 60, (n, 64)).astype(np.float64))


def test_forward_matches_oracle(gpu):
    import torch
    from paper_2311_17604_amd import pdd
    theta = _init(3, 0.3)
    X = _features(4, 1000)
    feat = torch.from_numpy(_f64_to_bits(X)).cuda()
    pdd.pred_set_weights(gpu, theta)
    got = pdd.pred_forward(gpu, feat).cpu().numpy().astype(np.float64)
    ref = mo.forward(theta.astype(np.float64), _bits_to_f64(feat), bf16_operands=True)[4]
    err = np.abs(got - ref)
    scale = 1.0 + np.abs(ref)
    assert np.median(err / scale) < 1e-4
    assert np.max(err / scale) < 5e-3


@pytest.mark.parametrize("n,tau", [(128, 0.9), (77, 0.5), (16, 0.75)])
def test_grad_matches_oracle(gpu, n, tau):
    import torch
    from paper_2311_17604_amd import pdd
    theta = _init(5 + n, 0.0)
    X = _features(6 + n, n)
    y = np.random.default_rng(7 + n).normal(0.5, 1.0, n).astype(np.float32)
    feat = torch.from_numpy(_f64_to_bits(X)).cuda()
    pdd.pred_set_weights(gpu, theta)
    g, loss = pdd.pred_grad(gpu, feat, torch.from_numpy(y).cuda(), tau)
    g = g.cpu().numpy().astype(np.float64)
    Xb = _bits_to_f64(feat)
    ref = mo.grad(theta.astype(np.float64), Xb, y.astype(np.float64), tau, bf16_operands=True)
    assert np.linalg.norm(g - ref) <= 1e-2 * np.linalg.norm(ref)
    # per block of the parameter vector
    for lo, hi in [(0, 4096), (4096, 4160), (4160, 8256), (8256, 8320), (8320, 8384), (8384, 8385)]:
        assert np.linalg.norm(g[lo:hi] - ref[lo:hi]) <= 2e-2 * np.linalg.norm(ref[lo:hi]) + 1e-6, (lo, hi)
    yhat = mo.forward(theta.astype(np.float64), Xb, bf16_operands=True)[4]
    r = y - yhat
    want_loss = np.mean(np.where(r > 0, tau * r, (tau - 1) * r))
    assert abs(loss - want_loss) <= 1e-3 * (1 + abs(want_loss))


def _training_rows(ctx, seeds, scale, k, b):
    import torch
    from paper_2311_17604_amd import pdd
    feats, tgts = [], []
    for s in seeds:
        w = scangen.config(1, scale=scale, seed=s)
        f, t = pdd.pred_samples(ctx, torch.from_numpy(w.xyz).cuda(), k, b)
        feats.append(f)
        tgts.append(t)
    return torch.cat(feats), torch.cat(tgts)


@pytest.fixture(scope="module")
def trained(gpu):
    """Predictor trained on k-NN radii (list width 16: k = 8, b = 8) of scans
    of the 200k-scan generator (other seeds); returns (parameters, losses)."""
    from paper_2311_17604_amd import pdd
    feat, tgt = _training_rows(gpu, [101, 102, 103, 104], 0.5, 8, 8)
    pdd.pred_set_weights(gpu, _init(11, float(tgt.mean().item())))
    losses = pdd.pred_train(gpu, feat, tgt, steps=1500, batch=128, lr=2e-3, tau=0.9, seed=5).cpu().numpy()
    return pdd.pred_get_weights(gpu), losses


def test_training_reduces_loss(trained):
    _, losses = trained
    assert np.all(np.isfinite(losses))
    assert losses[-100:].mean() < 0.6 * losses[:20].mean()


def test_predictor_gain_and_exactness(gpu, oracle_mod, trained):
    import torch
    from paper_2311_17604_amd import pdd
    params, _ = trained
    pdd.pred_set_weights(gpu, params)
    w = scangen.config(1, scale=0.7, seed=109)          # held out
    x = torch.from_numpy(w.xyz).cuda()
    pdd.pred_enable(gpu, False)
    plain = [t.cpu().numpy() for t in pdd.knn_cost(gpu, x, w.k, 8)]
    st_plain = gpu.stats()
    pdd.pred_enable(gpu, True, 0.25)
    pred = [t.cpu().numpy() for t in pdd.knn_cost(gpu, x, w.k, 8)]
    st_pred = gpu.stats()
    assert np.array_equal(plain[2], pred[2]) and np.array_equal(plain[1], pred[1])
    P = w.xyz.astype(np.int64)
    d_plain = ((P[plain[0]] - P[:, None, :]) ** 2).sum(-1)
    d_pred = ((P[pred[0]] - P[:, None, :]) ** 2).sum(-1)
    assert np.array_equal(d_plain, d_pred)
    # the gain: the predicted regions test fewer points, and most of them
    # certify their points' lists
    print("plain", st_plain, "learned", st_pred)
    assert st_pred["pred_hits"] > 4 * st_pred["pred_misses"]
    assert st_pred["knn_tested"] < st_plain["knn_tested"], (st_pred, st_plain)
    # and a decimation with the predictor on stays the oracle's
    small = scangen.config(1, scale=0.1, seed=110)
    ref = oracle_mod.decimate(small.xyz, small.k, small.keep, b=6)
    got = pdd.decimate(gpu, torch.from_numpy(small.xyz).cuda(), small.keep, small.k)
    gpu.stream.synchronize()
    pdd.pred_enable(gpu, False)
    for g_, r_, name in zip(got, ref, ("kept", "order", "order_cost")):
        g_ = g_.cpu().numpy()
        if name == "order_cost":
            g_ = g_.view(np.uint64)
        assert np.array_equal(g_, r_), name


def test_batch_with_predictor_equals_oracle(gpu, oracle_mod, trained):
    # the learned region inside a batched decimation (one segmented grid of
    # 12 scans): each scan's result is still the oracle's
    import torch
    from paper_2311_17604_amd import pdd
    params, _ = trained
    pdd.pred_set_weights(gpu, params)
    w = scangen.batch_config(12, scale=1 / 100, base_seed=10500)
    x = torch.from_numpy(w.xyz).cuda()
    pdd.pred_enable(gpu, True, 0.25)
    try:
        kept, order, oc = pdd.decimate_batch(gpu, x, w.offsets, w.keeps, w.k, b=8)
        gpu.stream.synchronize()
    finally:
        pdd.pred_enable(gpu, False)
    kept, order, oc = kept.cpu().numpy(), order.cpu().numpy(), oc.cpu().numpy().view(np.uint64)
    ko = np.concatenate([[0], np.cumsum(w.keeps)])
    ro = np.concatenate([[0], np.cumsum(np.diff(w.offsets) - w.keeps)])
    for s in range(len(w.keeps)):
        ref = oracle_mod.decimate(w.xyz[w.offsets[s]:w.offsets[s + 1]], w.k, int(w.keeps[s]), b=6)
        assert np.array_equal(kept[ko[s]:ko[s + 1]], ref[0]), ("kept", s)
        assert np.array_equal(order[ro[s]:ro[s + 1]], ref[1]), ("order", s)
        assert np.array_equal(oc[ro[s]:ro[s + 1]], ref[2]), ("order_cost", s)
