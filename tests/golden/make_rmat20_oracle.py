"""Write the oracle's reference for the RMAT scale-20 update stream.

Runs only the CPU oracle (oracle/) on the stream of
paper_2106_03824_amd.workloads.RmatStream(20, 16*2^20, seed=1, 16 build
batches, workload 2): the 16 insertion batches of the build, then rounds of
[10^6 insertions, 10^6 deletions, 10^6 mixed].  It stores the levels after
the build (int16) and, for every batch, a checksum of the levels and the
sweep/move counts, plus the oracle's single-core time per batch.

With ``resume R`` it starts from the stored post-build state (checked
against the stored digest of the last build batch) instead of rebuilding,
and writes the build batches' records back unchanged followed by R rounds;
rounds already in the stored trace must come out identical.

With the argument ``sizes`` it instead starts from the stored post-build
state (the build's edges and the levels above) and applies the batch sizes
10^4 and 10^5: insertions, then deletions, then mixed batches, with update
seeds 1000*2 + 100 + j for j = 100, 101, ...; the result goes to
rmat20_oracle_sizes.json.

    python tests/golden/make_rmat20_oracle.py [rounds | resume rounds | sizes]
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
OUT_SIZES = os.path.join(HERE, "rmat20_oracle_sizes.json")
SIZES = (10 ** 4, 10 ** 5)
SIZES_J0 = 100


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


def resume(rounds):
    st = W.RmatStream(SCALE, 16 * 2 ** SCALE, seed=1, build_batches=16, cfg=2)
    old = json.load(open(OUT_JSON))
    builds = [b for b in old["batches"] if b["kind"].startswith("build")]
    assert len(builds) == len(st.build)
    o = O.Oracle(st.n, 0.4, 3.0)
    lv0 = np.load(OUT_NPZ)["levels"].astype(np.int32)
    assert o.load_state(np.concatenate(st.build), lv0) == 0
    assert digest(o.levels()) == builds[-1]["sha"], "stored post-build levels do not match the trace"
    known = {b["kind"]: b for b in old["batches"]}
    trace = {"workload": old["workload"], "delta": 0.4, "lambda": 3.0, "batches": list(builds)}

    def record(kind, rc, dt):
        s = o.stats()
        item = {"kind": kind, "rc": rc, "seconds": round(dt, 3), "sha": digest(o.levels()),
                **{k: s[k] for k in ("applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up",
                                     "moves_down", "viol_ins0", "viol_del0")}}
        if kind in known:
            ref = {k: v for k, v in known[kind].items() if k != "seconds"}
            assert ref == {k: v for k, v in item.items() if k != "seconds"}, (kind, ref, item)
        trace["batches"].append(item)
        print(json.dumps(item), flush=True)
        tmp = OUT_JSON + ".tmp"
        json.dump(trace, open(tmp, "w"), indent=1)
        os.replace(tmp, OUT_JSON)

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


def sizes():
    st = W.RmatStream(SCALE, 16 * 2 ** SCALE, seed=1, build_batches=16, cfg=2)
    st.j = SIZES_J0
    o = O.Oracle(st.n, 0.4, 3.0)
    lv0 = np.load(OUT_NPZ)["levels"].astype(np.int32)
    assert o.load_state(np.concatenate(st.build), lv0) == 0
    trace = {"workload": "RMAT scale 20 after the 16 build batches (stored oracle levels); then insertions of "
                         "1e4 and 1e5, deletions of 1e4 and 1e5, mixed 1e4 and 1e5, update seeds from j=100",
             "delta": 0.4, "lambda": 3.0, "batches": []}
    plan = [("ins", c) for c in SIZES] + [("del", c) for c in SIZES] + [("mix", c) for c in SIZES]
    for kind, c in plan:
        if kind == "ins":
            args = (st.insert_batch(c), None)
        elif kind == "del":
            args = (None, st.delete_batch(c))
        else:
            args = st.mixed_batch(c)
        t = time.perf_counter()
        rc = o.update(*args)
        dt = time.perf_counter() - t
        s = o.stats()
        item = {"kind": f"{kind}{c}", "rc": rc, "seconds": round(dt, 3), "sha": digest(o.levels()),
                **{k: s[k] for k in ("applied_ins", "applied_del", "sweeps_ins", "sweeps_del", "moves_up",
                                     "moves_down", "viol_ins0", "viol_del0")}}
        trace["batches"].append(item)
        print(json.dumps(item), flush=True)
        json.dump(trace, open(OUT_SIZES, "w"), indent=1)
    assert o.check() == 0


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sizes":
        sizes()
    elif len(sys.argv) > 1 and sys.argv[1] == "resume":
        resume(int(sys.argv[2]))
    else:
        main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
