"""Write the oracle's reference for the RMAT scale-20 update stream.

Runs only the CPU oracle (oracle/) on the stream of
paper_2106_03824_amd.workloads.RmatStream(20, 16*2^20, seed=1, 16 build
batches, workload 2): the 16 insertion batches of the build, then rounds of
[10^6 insertions, 10^6 deletions, 10^6 mixed].  It stores the levels after
the build (int16) and, for every batch, a checksum of the levels and the
sweep/move counts, plus the oracle's single-core time per batch.

    python tests/golden/make_rmat20_oracle.py [rounds]
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

SCALE, BATCH = 20, 10 ** 6
OUT_NPZ = os.path.join(HERE, "rmat20_oracle_levels.npz")
OUT_JSON = os.path.join(HERE, "rmat20_oracle_trace.json")


def digest(levels):
    return hashlib.sha256(np.ascontiguousarray(levels, dtype=np.int32).tobytes()).hexdigest()[:32]


def main(rounds=2):
    st = W.RmatStream(SCALE, 16 * 2 ** SCALE, seed=1, build_batches=16, cfg=2)
    o = O.Oracle(st.n, 0.4, 3.0)
    trace = {"workload": "RMAT scale 20, 16*2^20 unique edges, seed 1, 16 build batches; then rounds of "
                         "[1e6 insert, 1e6 delete, 1e6 mixed]", "delta": 0.4, "lambda": 3.0, "batches": []}

    def record(kind, rc, dt):
        s = o.stats()
        lv = o.levels()
        item = {"kind": kind, "rc": rc, "seconds": round(dt, 3), "sha": digest(lv),
                **{k: s[k] for k in ("applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up",
                                     "moves_down", "viol_ins0", "viol_del0")}}
        trace["batches"].append(item)
        print(json.dumps(item), flush=True)
        json.dump(trace, open(OUT_JSON, "w"), indent=1)
        return lv

    for i, b in enumerate(st.build):
        t = time.perf_counter()
        rc = o.insert(b)
        lv = record(f"build{i}", rc, time.perf_counter() - t)
    assert o.check() == 0
    np.savez_compressed(OUT_NPZ, levels=lv.astype(np.int16))
    for r in range(rounds):
        ins = st.insert_batch(BATCH)
        t = time.perf_counter()
        rc = o.insert(ins)
        record(f"ins{r}", rc, time.perf_counter() - t)
        dele = st.delete_batch(BATCH)
        t = time.perf_counter()
        rc = o.delete(dele)
        record(f"del{r}", rc, time.perf_counter() - t)
        mi, md = st.mixed_batch(BATCH)
        t = time.perf_counter()
        rc = o.update(mi, md)
        record(f"mix{r}", rc, time.perf_counter() - t)
    assert o.check() == 0


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
