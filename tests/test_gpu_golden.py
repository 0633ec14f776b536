"""HIP path at the full workload sizes against the oracle's stored results.

tests/golden/oracle_hashes.json holds SHA-256 digests of the oracle's kept
indices, removal order and removal costs for each workload (written by
tests/golden/make_golden.py, which calls only the oracle and the input
generator).  The GPU runs in the default configuration that bench.py times.
Besides the digests, properties that hold at any size are checked: exact
keep count, ascending unique kept indices, kept and removed sets partition
the input, and the greedy's removal keys strictly decrease.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2311_17604_amd import scangen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
HASHES = os.path.join(HERE, "golden", "oracle_hashes.json")
# name -> (workload index, scale, crop), as in tests/golden/make_golden.py
WORKLOADS = {
    "scan-200k-k8-keep25": (1, 1.0, False),
    "scan-20M-k16-keep10@0.25": (2, 0.25, False),
    "scan-20M-k16-keep10": (2, 1.0, False),
}


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2311_17604_amd import pdd
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = pdd.Context(0)
    yield ctx
    ctx.close()


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_golden_workload(gpu, name):
    import torch
    from paper_2311_17604_amd import pdd
    ref = json.load(open(HASHES))[name]
    cfg, scale, crop = WORKLOADS[name]
    w = scangen.config(cfg, scale=scale, crop=crop)
    n = len(w.xyz)
    assert (n, w.k, w.keep) == (ref["n"], ref["k"], ref["keep"])
    x = torch.from_numpy(w.xyz).cuda()
    kept, order, oc = pdd.decimate(gpu, x, w.keep, w.k)
    gpu.stream.synchronize()
    kept = kept.cpu().numpy()
    order = order.cpu().numpy()
    oc = oc.cpu().numpy().view(np.uint64)
    # properties at any size
    assert len(kept) == w.keep and len(order) == n - w.keep
    assert np.all(np.diff(kept) > 0)
    seen = np.zeros(n, np.int32)
    np.add.at(seen, kept, 1)
    np.add.at(seen, order, 1)
    assert np.all(seen == 1)
    dec = (oc[1:] < oc[:-1]) | ((oc[1:] == oc[:-1]) & (order[1:] > order[:-1]))
    assert np.all(dec), "removal keys must strictly decrease"
    assert [int(v) for v in order[:8]] == ref["first_order"]
    assert int(oc[-1]) == ref["last_order_cost"]
    # the oracle's exact result
    assert _sha(kept.astype(np.int32)) == ref["kept_sha256"], "kept"
    assert _sha(order.astype(np.int32)) == ref["order_sha256"], "order"
    assert _sha(oc.astype(np.uint64)) == ref["order_cost_sha256"], "order_cost"
