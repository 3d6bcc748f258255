"""Write the oracle's static approximate k-core (Algorithm 6) of the RMAT-20
graph: the graph of paper_2106_03824_amd.workloads.RmatStream(20, 16*2^20,
seed=1), i.e. all its build batches, at the given eps values.  Stores, per
eps, the SHA-256 of the float64 estimates, the number of nonzero estimates,
the largest estimate and the oracle's single-core time (oracle only).

    python tests/golden/make_rmat20_static.py [eps ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.static_kcore as SKO  # noqa: E402
from paper_2106_03824_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "rmat20_static_oracle.json")


def main(eps_list):
    st = W.RmatStream(20, 16 * 2 ** 20, seed=1, build_batches=16, cfg=2)
    e = np.concatenate(st.build)
    out = json.load(open(OUT)) if os.path.exists(OUT) else {
        "workload": "RMAT scale 20, 16*2^20 unique edges, seed 1 (the RMAT-20 stream's graph after its build)",
        "estimates": {}}
    for eps in eps_list:
        t = time.perf_counter()
        est = SKO.static_approx_kcore(st.n, e, eps)
        dt = time.perf_counter() - t
        out["estimates"][repr(float(eps))] = {
            "sha": hashlib.sha256(np.ascontiguousarray(est, dtype=np.float64).tobytes()).hexdigest()[:32],
            "nonzero": int((est > 0).sum()), "max": float(est.max()), "seconds": round(dt, 1)}
        print(eps, out["estimates"][repr(float(eps))], flush=True)
        tmp = OUT + ".tmp"
        json.dump(out, open(tmp, "w"), indent=1)
        os.replace(tmp, OUT)


if __name__ == "__main__":
    main([float(x) for x in sys.argv[1:]] or [0.5, 1.0])
