"""Writes the oracle's results for the large workloads as SHA-256 digests
(kept, order, order_cost) to oracle_hashes.json beside this script.

Calls only the CPU oracle and the input generator.  Usage:
    python tests/golden/make_golden.py NAME [NAME ...]
NAME is one of the keys of WORKLOADS.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle  # noqa: E402
from paper_2311_17604_amd import scangen  # noqa: E402

OUT = os.path.join(HERE, "oracle_hashes.json")

# name -> (workload index, scale, crop); tests/test_gpu_golden.py repeats
# this table
WORKLOADS = {
    "scan-200k-k8-keep25": (1, 1.0, False),
    "scan-20M-k16-keep10@0.25": (2, 0.25, False),
    "scan-20M-k16-keep10": (2, 1.0, False),
    "merged-10st-500M-k8-keep5/crop3m": (3, 1.0, True),
    "merged-40st-2B-k8-keep2/crop3m": (5, 1.0, True),
}


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(names):
    for name in names:
        cfg, scale, crop = WORKLOADS[name]
        w = scangen.config(cfg, scale=scale, crop=crop)
        t = time.time()
        kept, order, oc = oracle.decimate(w.xyz, w.k, w.keep, b=8)
        dt = time.time() - t
        # re-read: several runs may write their workloads concurrently
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        data[name] = {
            "n": int(len(w.xyz)), "k": w.k, "keep": int(w.keep),
            "kept_sha256": digest(kept.astype(np.int32)),
            "order_sha256": digest(order.astype(np.int32)),
            "order_cost_sha256": digest(oc.astype(np.uint64)),
            "oracle_seconds": round(dt, 1), "oracle_cores": 1,
            "first_order": [int(v) for v in order[:8]],
            "last_order_cost": int(oc[-1]) if len(oc) else None,
        }
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(name, "done in %.1f s" % dt, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
