"""Write the oracle's reference for the RMAT scale-24 insertion stream.

Runs only the CPU oracle (oracle/) on the stream that the RMAT-24
benchmark and its GPU tests apply first: the R-MAT graph of scale 24 with
16*2^24 unique edges (a=0.57, b=0.19, c=0.19, seed 1), in the order of a
seeded random permutation (seed 3001), as insertion batches of 10^6 edges
from an empty graph.  For every batch it stores a checksum of the levels,
the sweep and move counts and the oracle's single-core time; the file is
rewritten after every batch, so a run stopped early leaves a valid prefix.

    python tests/golden/make_rmat24_oracle.py [max_batches]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2106_03824_amd import workloads as W  # noqa: E402

SCALE, BATCH, PERM_SEED = 24, 10 ** 6, 3001
OUT_JSON = os.path.join(HERE, "rmat24_oracle_trace.json")


def digest(levels):
    return hashlib.sha256(np.ascontiguousarray(levels, dtype=np.int32).tobytes()).hexdigest()[:32]


def main(max_batches):
    n, m0 = 2 ** SCALE, 16 * 2 ** SCALE
    t = time.perf_counter()
    perm = W.permute_edges(W.rmat(SCALE, m0, seed=1), PERM_SEED)
    print(f"generated in {time.perf_counter() - t:.1f}s", flush=True)
    o = O.Oracle(n, 0.4, 3.0)
    trace = {"workload": "RMAT scale 24, 16*2^24 unique edges, seed 1, permutation seed 3001, streamed as "
                         "insertion batches of 1e6 from an empty graph", "delta": 0.4, "lambda": 3.0, "batches": []}
    for i in range(min(max_batches, (m0 + BATCH - 1) // BATCH)):
        b = perm[i * BATCH:(i + 1) * BATCH]
        t = time.perf_counter()
        rc = o.insert(b)
        dt = time.perf_counter() - t
        s = o.stats()
        item = {"kind": f"stream{i}", "rc": rc, "seconds": round(dt, 3), "sha": digest(o.levels()),
                **{k: s[k] for k in ("applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up",
                                     "moves_down", "viol_ins0", "viol_del0", "top_level")}}
        trace["batches"].append(item)
        print(json.dumps(item), flush=True)
        tmp = OUT_JSON + ".tmp"
        json.dump(trace, open(tmp, "w"), indent=1)
        os.replace(tmp, OUT_JSON)
        assert rc == 0


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 30)
