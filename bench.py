#!/usr/bin/env python3
"""Edge updates/s of the batch-dynamic PLDS on one MI355X.

Default workload: an R-MAT graph of scale 24 (2^24
vertices, 16*2^24 unique edges, a=0.57 b=0.19 c=0.19, seed 1), delta=0.4,
lambda=3, in the order of a seeded random permutation (seed 3001).  All but
a held-out tail of the permutation is streamed in as insertion batches of
10^6 (the build, not timed; its rate is reported, and its first batches are
checked against the stored oracle trace of the stream).  One step applies
three batches of 10^6 updates each through the C ABI: the next 10^6 tail
edges (insertions), 10^6 edges sampled without replacement from the built
graph (deletions), and a mixed batch of half each.  Batches are in HBM
before the timed region; the value is the number of applied updates over the
wall time of the K timed steps.

Beside it: the RMAT-20 stream (16 build batches, then
rounds of 10^6 new uniform pairs, sampled deletions and mixed batches, every
batch checked against the stored oracle trace of the stream; --no-rmat20
leaves it out), the insertion-scan kernel against the HBM roofline (its
launches timed with HIP events inside the library, on the call's stream;
HBM traffic per launch from the committed counter summary under profiles/
when it matches the current kernel source), the CPU oracle (one core)
timed on a bounded sample of the same RMAT-24 stream, and, as extra keys,
the batched form ("batched", as --batched below; --no-batched leaves it
out) and the serving form ("serving", as --serve below; --no-serve).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --workload rmat20      # the RMAT-20 stream alone
    python bench.py --workload stream [--scale 24] [--batch 1000000]
                       # the whole graph streamed in insertion batches, then
                       # two deletion batches and one mixed batch, all timed

With --batched it runs the batched form instead: 256 independent graphs of
uneven size (128 Erdos-Renyi G(n, p) with n log-uniform in [2^10, 2^16] and
mean degree uniform in [4, 32]; 128 R-MAT graphs with scale uniform in
[10, 16] and edge factor 8), each built by one insertion batch, then one
measured batch per graph (insertion or deletion with probability 1/2, size
uniform in [10^3, 5*10^4], deletions clamped to m).  The measured batches
of all graphs go through one multi-graph handle in one call (the value), and
through one plain handle per graph in a loop; the levels of both must be
identical.  Before measuring, the launch schedule of the multi-graph handle
is searched (paper_2106_03824_amd/autotune.py) on a second batch per graph
drawn with other seeds; the fused call is timed under the default schedule
and under the one found, each from the post-build state, median of --steps
runs.

    python bench.py --batched [--tune-record search.json]

With --serve it runs the serving form: 64 resident R-MAT graphs (scale
uniform in [16, 22], edge factor 16) behind the continuous-batching server
of paper_2106_03824_amd/serve.py (shards of --slots graphs, each a
multi-graph handle; a shard pass serves the pending requests of distinct
graphs with one fused update call and one coreness call).  Request streams
(half update batches of log-uniform size in [10^2, 10^6], 70% insertions;
half coreness queries of 10^3 vertices) are served first all at once (the
saturation rate), then as Poisson streams at 10%, 50%, 90% and 120% of it;
p50/p99 latency per rate.  Afterwards the same graphs and requests are
served one at a time with a plain handle per graph, and every query result
and final level must be identical.

    python bench.py --serve [--serve-scales 16 22] [--serve-graphs 64]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edge updates/sec (ins, del) at 1e6 batch"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 2 << 30
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_ins_scan_rmat20_hbm_counters.txt")
PROFILE_SUMMARY_24 = os.path.join(ROOT, "profiles", "k_ins_scan_rmat24_hbm_counters.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2106_03824_amd", "csrc", "plds.hip")


def source_digest():
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()[:16]


def measured_traffic(summary=None):
    """HBM bytes per k_ins_scan launch from the committed counter summary, if
    it was taken on the current kernel source; else None."""
    summary = summary or PROFILE_SUMMARY
    if not os.path.exists(summary):
        return None
    vals = {}
    for line in open(summary):
        if ":" in line and not line.startswith(" "):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
TRACE = os.path.join(ROOT, "tests", "golden", "rmat20_oracle_trace.json")
LEVELS = os.path.join(ROOT, "tests", "golden", "rmat20_oracle_levels.npz")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def digest(levels):
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(levels, dtype=np.int32).tobytes()).hexdigest()[:32]


def cpu_baseline(build_edges, n, seconds_target):
    """The oracle, single-threaded, on a bounded sample of the same stream:
    from the stored post-build oracle state, one 1e6 deletion batch and one
    1e6 mixed batch (half new pairs, half sampled edges) drawn from the
    post-build graph with the stream's generators."""
    import numpy as np
    import oracle as O
    from paper_2106_03824_amd import workloads as W
    if not os.path.exists(LEVELS):
        return None
    lv = np.load(LEVELS)["levels"].astype(np.int32)
    o = O.Oracle(n, 0.4, 3.0)
    t = time.perf_counter()
    rc = o.load_state(build_edges, lv)
    load_s = time.perf_counter() - t
    if rc != 0:
        log("oracle rejected the stored state", rc)
        return None
    dele = W.sample_edges(build_edges, 10 ** 6, 2900)
    t = time.perf_counter()
    assert o.delete(dele) == 0
    t_del = time.perf_counter() - t
    u_del = o.stats()["applied_del"]
    rest = o.edges()
    mi = W.new_pairs(n, rest, 5 * 10 ** 5, 2901)
    md = W.sample_edges(rest, 5 * 10 ** 5, 2902)
    t = time.perf_counter()
    assert o.update(mi, md) == 0
    t_mix = time.perf_counter() - t
    s = o.stats()
    u_mix = s["applied_ins"] + s["applied_del"]
    total = t_del + t_mix
    return {"value": (u_del + u_mix) / total, "unit": "edge updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (one core) loaded with the stored post-build oracle state of this RMAT-20 stream "
                      f"(load {load_s:.1f}s, not timed); one 1e6 deletion batch ({t_del:.2f}s) and one 1e6 "
                      f"mixed batch ({t_mix:.1f}s) drawn from the post-build graph; a 1e6 insertion batch "
                      f"(over 2 min on the oracle) is left out of the sample",
            "rates": {"del": u_del / t_del, "mix": u_mix / t_mix}}


def _baseline(value, unit, t_work, sample, **extra):
    out = {"value": value, "unit": unit, "cores": 1, "kind": "oracle", "sample": sample,
           "seconds": round(t_work, 2)}
    out.update(extra)
    return out


def cpu_baseline_opt(st, n, lpg=-1, coeff=0.0, jump=False, seconds=20.0):
    """The oracle in the same variant (PLDSOpt levels, coefficient, jumps;
    one core) on the start of the same RMAT-20 stream: its build edges in
    insertion batches of 1e5 until `seconds` have passed (a build batch of
    1e6 takes the oracle minutes at the default level structure)."""
    import oracle as O
    o = O.Oracle(n, 0.4, 3.0, lpg, coeff=coeff, jump=jump)
    e = st.build[0]
    C = 10 ** 5
    u, dt, off = 0, 0.0, 0
    while dt < seconds and off + C <= len(e):
        t = time.perf_counter()
        assert o.insert(e[off:off + C]) == 0
        dt += time.perf_counter() - t
        u += o.stats()["applied_ins"]
        off += C
        log(f"cpu baseline: {off} edges in {dt:.1f}s")
    return _baseline(u / dt, "edge updates/s", dt,
                     f"oracle (one core) in the same variant (levels per group {lpg}, coefficient "
                     f"{coeff or '2+3/lambda'}, jumps {bool(jump)}), the stream's first {off} build edges as "
                     f"insertion batches of 1e5 (the oracle has no stored post-build state for the variants)")


def cpu_baseline_static(eps):
    """Algorithm 6's oracle (one core) on the RMAT-19 graph of the same
    generator and edge factor (the RMAT-20 run takes it about 50 s; its cost
    is linear in m per peel round)."""
    import oracle.static_kcore as SKO
    from paper_2106_03824_amd import workloads as W
    scale = 19
    e = W.rmat(scale, 16 * 2 ** scale, seed=1)
    t = time.perf_counter()
    SKO.static_approx_kcore(2 ** scale, e, eps)
    dt = time.perf_counter() - t
    return _baseline(len(e) / dt, "edges/s", dt,
                     f"oracle (one core), Algorithm 6 at eps={eps} on the RMAT-19 graph of the same generator "
                     f"and edge factor ({len(e)} edges); the RMAT-20 graph takes it about 50 s")


def cpu_baseline_vertex(build_edges, n, vertex_batches, warmup):
    """The oracle (one core) from the stored post-build state of the RMAT-20
    stream, deleting the same vertex batches as the timed run (the warm-up
    batches first, untimed)."""
    import numpy as np
    import oracle as O
    import oracle.vertex as OV
    if not os.path.exists(LEVELS):
        return None
    lv = np.load(LEVELS)["levels"].astype(np.int32)
    o = O.Oracle(n, 0.4, 3.0)
    if o.load_state(build_edges, lv) != 0:
        return None
    edges, secs = 0, 0.0
    for i, vs in enumerate(vertex_batches):
        m0 = o.m
        t = time.perf_counter()
        assert OV.delete_vertices(o, vs) == 0
        dt = time.perf_counter() - t
        if i >= warmup:
            edges += m0 - o.m
            secs += dt
    return _baseline(edges / secs, "edges/s", secs,
                     f"oracle (one core) loaded with the stored post-build state (load not timed), deleting the "
                     f"timed run's {len(vertex_batches) - warmup} batches of 1e4 vertices after its warm-up batch; "
                     f"the renumbering rebuild is left out")


def cpu_baseline_orient():
    """The oracle (one core) on the same stream recipe at RMAT-14 (batches
    of 2^14, the 1:16 batch-to-graph ratio of the RMAT-20 run): one round of
    insertion, deletion and mixed batches, each with its flips F and
    oriented updates J; the build is not timed.  The oracle's F and J are
    linear in m per batch (a 1e6 batch on RMAT-20 takes it over 3 minutes)."""
    import oracle as O
    import oracle.orient as OR
    from paper_2106_03824_amd import workloads as W
    scale, B = 14, 2 ** 14
    st = W.RmatStream(scale, 16 * 2 ** scale, seed=1, build_batches=16, cfg=2)
    o = O.Oracle(st.n, 0.4, 3.0)
    for b in st.build:
        assert o.insert(b) == 0
    u, secs = 0, 0.0
    for kind in ("ins", "del", "mix"):
        if kind == "ins":
            ins, dele = st.insert_batch(B), None
        elif kind == "del":
            ins, dele = None, st.delete_batch(B)
        else:
            ins, dele = st.mixed_batch(B)
        lv0, e0 = o.levels(), o.edges()
        t = time.perf_counter()
        assert o.update(ins, dele) == 0
        s = o.stats()
        lv1, e1 = o.levels(), o.edges()
        OR.flips(lv0, lv1, e0, e1)
        a_ins, a_del = OR.applied_updates(e0, ins, dele)
        OR.oriented_updates(lv0, lv1, a_ins, a_del)
        secs += time.perf_counter() - t
        u += s["applied_ins"] + s["applied_del"]
    return _baseline(u / secs, "edge updates/s", secs,
                     f"oracle (one core) on the same stream recipe at RMAT-14 (build not timed): one round of "
                     f"{B}-update insertion, deletion and mixed batches, each with F and J (batch:graph 1:16 as "
                     f"in the RMAT-20 run, whose F and J take the oracle over 3 minutes per batch)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24", choices=["rmat24", "rmat20", "stream"],
                    help="rmat24 (default): the RMAT-24 stream and timed rounds of ins/del/mix, "
                         "with the RMAT-20 stream reported beside it; rmat20: that stream alone; "
                         "stream: the whole RMAT graph of --scale streamed in insertion batches, then deletions")
    ap.add_argument("--scale", type=int, default=24, help="scale of the rmat24 and stream workloads")
    ap.add_argument("--no-rmat20", action="store_true", help="leave the RMAT-20 stream out of the default run")
    ap.add_argument("--no-batched", action="store_true", help="leave the batched form out of the default run")
    ap.add_argument("--no-serve", action="store_true", help="leave the serving form out of the default run")
    ap.add_argument("--batch", type=int, default=10 ** 6)
    ap.add_argument("--kernel", default="ins_scan", help="kernel timed for the roofline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 2 GiB (reference for the HBM byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched", action="store_true", help="the batched form: 256 graphs in one handle")
    ap.add_argument("--graphs", type=int, default=256)
    ap.add_argument("--tune-reps", type=int, default=3,
                    help="timed runs per schedule of the batched search (0: no search, default schedule)")
    ap.add_argument("--tune-record", default=None, help="where the batched form writes its schedule search (JSON)")
    ap.add_argument("--serve", action="store_true", help="the serving form: resident graphs behind a request loop")
    ap.add_argument("--opt", action="store_true",
                    help="the default RMAT-20 stream with the PLDSOpt level structure (ceil(log_{1+delta} n / 50) "
                         "levels per group)")
    ap.add_argument("--jump", action="store_true",
                    help="the RMAT-20 stream with the implementation's insertion procedure (upward desire-level jumps)")
    ap.add_argument("--coeff", type=float, default=0.0,
                    help="the RMAT-20 stream with this Invariant-1 coefficient in place of 2+3/lambda (1.1: the "
                         "paper's heuristic parameters)")
    ap.add_argument("--static", action="store_true",
                    help="the static approximate k-core (Algorithm 6) of the RMAT-20 graph after the build")
    ap.add_argument("--static-eps", type=float, nargs="+", default=[0.5, 1.0, 0.1])
    ap.add_argument("--vertex", action="store_true",
                    help="vertex deletions (1e4 vertices per batch) and a renumbering rebuild on the RMAT-20 graph")
    ap.add_argument("--orient", action="store_true",
                    help="the RMAT-20 stream with the orientation outputs (flips F, oriented updates J) per batch")
    ap.add_argument("--serve-graphs", type=int, default=64)
    ap.add_argument("--serve-scales", type=int, nargs=2, default=[16, 22])
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--slots", type=int, default=8, help="graph slots per shard of the serving form")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the structure is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2106_03824_amd import plds as P
    from paper_2106_03824_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": COPY_BYTES, "note": "one device-to-device copy kernel, read+write"}))
        return
    dev = torch.device("cuda", 0)
    if args.batched:
        print(json.dumps(run_batched(args, P, W, torch, np)), flush=True)
        return
    if args.serve:
        print(json.dumps(run_serve(args, P, W, torch, np)), flush=True)
        return
    if args.orient:
        return run_orient(args, P, W, torch, np)
    if args.static:
        return run_static(args, P, W, torch, np)
    if args.vertex:
        return run_vertex(args, P, W, torch, np)
    if args.workload == "stream":
        return run_stream(args, P, W, torch, np)
    if args.opt or args.jump or args.coeff or args.workload == "rmat20":
        out = run_rmat20(args, P, W, torch, np, args.steps, args.warmup)
        print(json.dumps(out), flush=True)
        return
    return run_rmat24(args, P, W, torch, np)


def run_rmat20(args, P, W, torch, np, steps, warmup):
    """The RMAT-20 stream (16 build batches, then rounds of
    1e6 insertions, deletions and mixed updates), checked against the stored
    oracle trace; returns the JSON object."""
    dev = torch.device("cuda", 0)
    scale, B = 20, 10 ** 6
    m0 = 16 * 2 ** scale
    log("generating R-MAT", scale, m0)
    st = W.RmatStream(scale, m0, seed=1, build_batches=16, cfg=2)
    n = st.n
    lpg = P.PLDS_LPG_OPT if args.opt else 0
    variant = args.opt or args.jump or args.coeff
    kernel = "jmp_scan" if args.jump and args.kernel == "ins_scan" else args.kernel
    g = P.PLDS(n, 0.4, 3.0, lpg, 2 * m0, up_coeff=args.coeff, up_jump=args.jump)
    # the stored oracle trace is of the paper's level structure
    trace = json.load(open(TRACE)) if (scale == 20 and B == 10 ** 6 and not variant and os.path.exists(TRACE)) \
        else None
    parity = {"batches_checked": 0, "mismatches": 0}

    def check(idx, lv=None, s=None):
        if trace is None or idx >= len(trace["batches"]):
            return
        ref = trace["batches"][idx]
        lv = g.levels().cpu().numpy() if lv is None else lv
        ok = digest(lv) == ref["sha"]
        s = g.stats() if s is None else s
        for k in ("sweeps_ins", "sweeps_del", "moves_up", "moves_down", "applied_ins", "applied_del"):
            ok = ok and s[k] == ref[k]
        parity["batches_checked"] += 1
        parity["mismatches"] += 0 if ok else 1
        if not ok:
            log("PARITY MISMATCH at batch", idx, ref["kind"])

    t_build = time.perf_counter()
    idx = 0
    build_updates = 0
    for i, b in enumerate(st.build):
        e = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
        P.plds_batch_insert(g.h, e)
        build_updates += g.stats()["applied_ins"]
        check(idx)
        idx += 1
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t_build
    log(f"build: {build_updates} edges in {t_build:.2f}s")

    rounds = warmup + steps
    batches = []
    for r in range(rounds):
        ins = st.insert_batch(B)
        dele = st.delete_batch(B)
        mi, md = st.mixed_batch(B)
        batches.append([("ins", torch.from_numpy(ins).to(dev), None),
                        ("del", None, torch.from_numpy(dele).to(dev)),
                        ("mix", torch.from_numpy(mi).to(dev), torch.from_numpy(md).to(dev))])
    torch.cuda.synchronize()
    log("batches ready")

    per_kind = {"ins": [0, 0.0], "del": [0, 0.0], "mix": [0, 0.0]}
    lat = []
    tot = {"updates": 0, "alg_bytes": 0, "timed_ms": 0.0, "launches": 0, "sweeps": 0, "moves": 0}
    snaps = []          # (batch index, device copy of the levels, stats) for the parity check after timing
    for r in range(rounds):
        timed = r >= warmup
        if timed and r == warmup:
            P.plds_set_timing(g.h, kernel)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for kind, ins, dele in batches[r]:
            tb = time.perf_counter()
            P.plds_update(g.h, ins, dele)
            dt = time.perf_counter() - tb
            s = g.stats()
            if timed:
                u = s["applied_ins"] + s["applied_del"]
                per_kind[kind][0] += u
                per_kind[kind][1] += dt
                lat.append(dt)
                tot["updates"] += u
                tot["alg_bytes"] += kernel_bytes(kernel, s)
                tot["timed_ms"] += s["timed_ms"]
                tot["launches"] += s["timed_launches"]
                tot["sweeps"] += s["sweeps_ins"] + s["sweeps_del"]
                tot["moves"] += s["moves_up"] + s["moves_down"]
                snaps.append((idx, g.levels(), s))
                log(f"batch {idx} {kind}: {u} updates in {dt * 1e3:.2f} ms, sweeps {s['sweeps_ins'] + s['sweeps_del']}, "
                    f"host syncs {s['host_syncs']}")
            else:
                check(idx)
            idx += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.plds_set_timing(g.h, 0)
    wall = t1 - t0
    value = tot["updates"] / wall
    log(f"timed: {tot['updates']} updates in {wall:.3f}s -> {value:.3e}/s")
    for i, lv, s in snaps:
        check(i, lv.cpu().numpy(), s)

    roof = None
    if tot["launches"] > 0 and tot["timed_ms"] > 0:
        avg_ms = tot["timed_ms"] / tot["launches"]
        per_launch = tot["alg_bytes"] / tot["launches"]
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic() if kernel == "ins_scan" and not variant else None,
                "kernel": "k_" + kernel,
                "avg_launch_us": round(avg_ms * 1e3, 3), "launches": tot["launches"],
                "alg_bytes_per_launch": round(per_launch, 1)}
    lat_ms = sorted(x * 1e3 for x in lat)
    out = {
        "metric": METRIC, "value": value, "unit": "edge updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": wall / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16-build16-then-ins/del/mix-{B}" + ("-pldsopt" if args.opt else "")
                   + ("-jump" if args.jump else "") + (f"-coeff{args.coeff}" if args.coeff else ""),
                   "n": n, "m0": m0, "delta": 0.4, "lambda": 3.0, "levels_per_group": g.L, "batch": B,
                   "step": "1 insertion + 1 deletion + 1 mixed batch"},
        "rates": {k: (v[0] / v[1] if v[1] else None) for k, v in per_kind.items()},
        "batch_latency_ms": {"p50": lat_ms[len(lat_ms) // 2], "p99": lat_ms[min(len(lat_ms) - 1,
                                                                              int(0.99 * len(lat_ms)))]},
        "sweeps_per_step": tot["sweeps"] / steps, "moves_per_step": tot["moves"] / steps,
        "build_updates_per_s": build_updates / t_build,
        "roofline": roof,
        "parity_vs_oracle_trace": parity if trace is not None else None,
    }
    if variant:
        out["invariants_hold"] = g.check() == 0   # no stored oracle trace for these variants
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_opt(st, n, lpg, args.coeff, args.jump)
    elif not args.no_cpu_baseline and args.workload == "rmat20":
        out["cpu_baseline"] = cpu_baseline(st_edges_after_build(st), n, args.cpu_seconds)
    g.close()
    return out


RMAT24_TRACE = os.path.join(ROOT, "tests", "golden", "rmat24_oracle_trace.json")
PERM_SEED_24 = 3001   # permutation of the RMAT-24 stream (as in tests/golden/make_rmat24_oracle.py)


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def cpu_baseline_rmat24(perm, n, seconds):
    """The oracle (one core) on the same RMAT-24 stream, from its start (the
    post-build state of 2.3e8 edges is out of its reach in the time given):
    the stream's first edges as insertion batches of 1e5 until half the
    budget is spent, then one deletion batch of 1e5 edges sampled from those
    and one mixed batch (5e4 next stream edges, 5e4 sampled)."""
    import numpy as np
    import oracle as O
    from paper_2106_03824_amd import workloads as W
    o = O.Oracle(n, 0.4, 3.0)
    C = 10 ** 5
    u_ins = off = 0
    t_ins = 0.0
    while t_ins < seconds / 2 and off + C <= len(perm) // 2:
        t = time.perf_counter()
        assert o.insert(perm[off:off + C]) == 0
        t_ins += time.perf_counter() - t
        u_ins += o.stats()["applied_ins"]
        off += C
    dele = W.sample_edges(perm[:off], C, 3200)
    t = time.perf_counter()
    assert o.delete(dele) == 0
    t_del = time.perf_counter() - t
    u_del = o.stats()["applied_del"]
    rest = o.edges()
    mi, md = perm[off:off + C // 2], W.sample_edges(rest, C // 2, 3201)
    t = time.perf_counter()
    assert o.update(mi, md) == 0
    t_mix = time.perf_counter() - t
    s = o.stats()
    u_mix = s["applied_ins"] + s["applied_del"]
    total = t_ins + t_del + t_mix
    out = {"value": (u_ins + u_del + u_mix) / total, "unit": "edge updates/s", "cores": 1, "kind": "oracle",
           "sample": f"oracle (one core, single-threaded) on the RMAT-24 stream from its start: the first {off} "
                     f"permuted edges as insertion batches of 1e5 ({t_ins:.1f}s), one 1e5 deletion batch sampled "
                     f"from them ({t_del:.2f}s) and one 1e5 mixed batch ({t_mix:.2f}s); the GPU's timed batches "
                     f"run against the 2.3e8-edge graph, which the oracle cannot reach in this budget",
           "rates": {"ins": u_ins / t_ins, "del": u_del / t_del, "mix": u_mix / t_mix}, "seconds": round(total, 2)}
    out.update(cpu_info())
    return out


def run_rmat24(args, P, W, torch, np):
    """R-MAT of scale 24 (16*2^24 unique edges, seed 1) in the
    order of a seeded random permutation.  All but a held-out tail of the
    permutation is streamed in as insertion batches of 1e6 (the build; its
    first batches are checked against the stored oracle trace of the stream),
    then each of the W + K rounds applies 1e6 insertions (the next tail
    edges), 1e6 deletions (sampled without replacement from the built graph)
    and a mixed batch (5e5 tail edges, 5e5 sampled deletions)."""
    scale, B = args.scale, args.batch
    n, m0 = 2 ** scale, 16 * 2 ** scale
    R = args.warmup + args.steps
    per_round_ins = B + (B - B // 2)
    hold = R * per_round_ins
    if hold >= m0 // 2:
        raise SystemExit("too many rounds for the graph: the held-out tail would exceed half of it")
    t = time.perf_counter()
    e = W.rmat(scale, m0, seed=1)
    perm = W.permute_edges(e, PERM_SEED_24)
    del e
    nb = m0 - hold
    dels = W.sample_edges(perm[:nb], R * (B + B // 2), PERM_SEED_24 + 99)
    log(f"R-MAT {scale}: {m0} edges, build {nb}, held out {hold}, in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda", 0)
    perm_d = torch.from_numpy(perm).to(dev)
    dels_d = torch.from_numpy(dels).to(dev)
    trace = None
    if scale == 24 and B == 10 ** 6 and os.path.exists(RMAT24_TRACE):
        trace = json.load(open(RMAT24_TRACE))["batches"]
    g = P.PLDS(n, 0.4, 3.0, 0, 2 * m0)
    parity = {"batches_checked": 0, "mismatches": 0, "trace_batches": len(trace) if trace else 0}
    torch.cuda.synchronize()
    t_build = time.perf_counter()
    build_updates, build_sweeps = 0, []
    for i, off in enumerate(range(0, nb, B)):
        P.plds_update(g.h, perm_d[off:min(off + B, nb)], None)
        s = g.stats()
        build_updates += s["applied_ins"]
        build_sweeps.append(s["sweeps_ins"])
        if trace is not None and i < len(trace):
            ref = trace[i]
            ok = digest(g.levels().cpu().numpy()) == ref["sha"] and all(
                s[k] == ref[k] for k in ("applied_ins", "sweeps_ins", "moves_up", "viol_ins0"))
            parity["batches_checked"] += 1
            parity["mismatches"] += 0 if ok else 1
            if not ok:
                log("PARITY MISMATCH at stream batch", i)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t_build
    log(f"build: {build_updates} edges in {t_build:.2f}s ({parity['batches_checked']} batches checked)")

    def rnd(r):
        a = nb + r * per_round_ins
        d = r * (B + B // 2)
        return [("ins", perm_d[a:a + B], None), ("del", None, dels_d[d:d + B]),
                ("mix", perm_d[a + B:a + per_round_ins], dels_d[d + B:d + B + B // 2])]

    per_kind = {"ins": [0, 0.0], "del": [0, 0.0], "mix": [0, 0.0]}
    lat = []
    tot = {"updates": 0, "alg_bytes": 0, "timed_ms": 0.0, "launches": 0, "sweeps": 0, "moves": 0, "syncs": 0,
           "calls": 0, "ins_steps": 0, "ins_loop_steps": 0, "ins_loop_launches": 0}
    t0 = None
    for r in range(R):
        timed = r >= args.warmup
        if timed and r == args.warmup:
            P.plds_set_timing(g.h, args.kernel)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for kind, ins, dele in rnd(r):
            tb = time.perf_counter()
            P.plds_update(g.h, ins, dele)
            dt = time.perf_counter() - tb
            s = g.stats()
            if timed:
                u = s["applied_ins"] + s["applied_del"]
                per_kind[kind][0] += u
                per_kind[kind][1] += dt
                lat.append(dt)
                tot["updates"] += u
                tot["alg_bytes"] += kernel_bytes(args.kernel, s)
                tot["timed_ms"] += s["timed_ms"]
                tot["launches"] += s["timed_launches"]
                tot["sweeps"] += s["sweeps_ins"] + s["sweeps_del"]
                tot["moves"] += s["moves_up"] + s["moves_down"]
                tot["syncs"] += s["host_syncs"]
                tot["calls"] += 1
                for f in ("ins_steps", "ins_loop_steps", "ins_loop_launches"):
                    tot[f] += s[f]
                log(f"round {r} {kind}: {u} updates in {dt * 1e3:.2f} ms, sweeps {s['sweeps_ins'] + s['sweeps_del']}, "
                    f"host syncs {s['host_syncs']}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.plds_set_timing(g.h, 0)
    value = tot["updates"] / wall
    log(f"timed: {tot['updates']} updates in {wall:.3f}s -> {value:.3e}/s")
    check = g.check()
    info = g.info()
    g.close()
    del perm_d, dels_d
    torch.cuda.empty_cache()
    roof = roofline(tot, args.kernel)
    if roof is not None and args.kernel == "ins_scan":
        roof["traffic"] = measured_traffic(PROFILE_SUMMARY_24)
    lat_ms = sorted(x * 1e3 for x in lat)
    out = {
        "metric": METRIC, "value": value, "unit": "edge updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16-stream{B}-then-ins/del/mix-{B}", "n": n, "m0": m0,
                   "built_edges": nb, "delta": 0.4, "lambda": 3.0, "levels_per_group": info["L"], "K": info["K"],
                   "batch": B,
                   "step": "1 insertion (held-out stream edges) + 1 deletion (sampled) + 1 mixed batch"},
        "rates": {k: (v[0] / v[1] if v[1] else None) for k, v in per_kind.items()},
        "batch_latency_ms": {"p50": lat_ms[len(lat_ms) // 2],
                             "p99": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))]},
        "sweeps_per_step": tot["sweeps"] / args.steps, "moves_per_step": tot["moves"] / args.steps,
        "host_syncs_per_call": tot["syncs"] / max(tot["calls"], 1),
        "insertion_steps_per_step": {"all": tot["ins_steps"] / args.steps,
                                     "single_block_loop": tot["ins_loop_steps"] / args.steps,
                                     "loop_launches": tot["ins_loop_launches"] / args.steps},
        "build": {"edges": build_updates, "seconds": round(t_build, 3), "updates_per_s": build_updates / t_build,
                  "batches": len(build_sweeps), "sweeps_per_batch": float(np.mean(build_sweeps)),
                  "parity_vs_oracle_trace": parity},
        "roofline": roof,
        "device_check": check,
    }
    if not args.no_rmat20:
        r20 = run_rmat20(args, P, W, torch, np, min(args.steps, 20), min(args.warmup, 5))
        out["rmat20"] = {k: r20[k] for k in ("value", "steps", "warmup", "ms_per_step", "rates", "batch_latency_ms",
                                             "sweeps_per_step", "roofline", "parity_vs_oracle_trace", "config")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_rmat24(perm, n, args.cpu_seconds)
    del perm
    if not args.no_batched:   # the batched form, as extra keys
        b = run_batched(args, P, W, torch, np)
        out["batched"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "per_graph_loop", "default_schedule",
                                            "schedule", "schedules_timed", "speedup_vs_loop", "identical_levels",
                                            "level_steps", "level_steps_alone", "config")}
    if not args.no_serve:     # the serving form, as extra keys
        v = run_serve(args, P, W, torch, np)
        out["serving"] = {k: v[k] for k in ("value", "unit", "latency", "identical_to_alone", "errors",
                                            "one_at_a_time", "config")}
    print(json.dumps(out), flush=True)


def kernel_bytes(kernel, s):
    """Algorithmic bytes of one call moved by the timed kernel: the insertion
    scan kernel and the single-block loop of small insertion steps split the
    up-moves' bytes between them."""
    if kernel == "ins_scan":
        return s["alg_bytes_up"] - s["alg_bytes_up_loop"]
    if kernel == "ins_loop":
        return s["alg_bytes_up_loop"]
    return s["alg_bytes_up"]


def roofline(tot, kernel):
    if tot["launches"] <= 0 or tot["timed_ms"] <= 0:
        return None
    avg_ms = tot["timed_ms"] / tot["launches"]
    per_launch = tot["alg_bytes"] / tot["launches"]
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_" + kernel,
            "avg_launch_us": round(avg_ms * 1e3, 3), "launches": tot["launches"],
            "alg_bytes_per_launch": round(per_launch, 1)}


def run_stream(args, P, W, torch, np):
    """Large streamed workload: build by timed insertion batches, then
    deletion and mixed batches, all timed."""
    scale, B = args.scale, args.batch
    n, m0 = 2 ** scale, 16 * 2 ** scale
    t = time.perf_counter()
    e = W.rmat(scale, m0, seed=1)
    log(f"R-MAT {scale}: {m0} edges in {time.perf_counter() - t:.1f}s")
    perm = W.permute_edges(e, 1000 * 3 + 1)
    dels = W.sample_edges(e, 2 * B + B // 2, 1000 * 3 + 100)
    mix_ins = W.new_pairs(n, e, B - B // 2, 1000 * 3 + 101)
    del e
    dev = torch.device("cuda", 0)
    perm_d = torch.from_numpy(perm).to(dev)
    del perm
    dels_d = torch.from_numpy(dels).to(dev)
    mix_ins_d = torch.from_numpy(mix_ins).to(dev)
    plan = [("ins", perm_d[i:i + B], None) for i in range(0, m0, B)]
    plan += [("del", None, dels_d[:B]), ("del", None, dels_d[B:2 * B]), ("mix", mix_ins_d, dels_d[2 * B:])]
    g = P.PLDS(n, 0.4, 3.0, 0, 2 * m0)
    log(f"batches ready: {len(plan)}")
    P.plds_set_timing(g.h, args.kernel)
    per_kind = {"ins": [0, 0.0], "del": [0, 0.0], "mix": [0, 0.0]}
    tot = {"updates": 0, "alg_bytes": 0, "timed_ms": 0.0, "launches": 0}
    sweeps, lat = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (kind, ins, dele) in enumerate(plan):
        tb = time.perf_counter()
        P.plds_update(g.h, ins, dele)
        dt = time.perf_counter() - tb
        s = g.stats()
        u = s["applied_ins"] + s["applied_del"]
        per_kind[kind][0] += u
        per_kind[kind][1] += dt
        lat.append(dt)
        tot["updates"] += u
        tot["alg_bytes"] += kernel_bytes(args.kernel, s)
        tot["timed_ms"] += s["timed_ms"]
        tot["launches"] += s["timed_launches"]
        sweeps.append(s["sweeps_ins"] + s["sweeps_del"])
        if i % 16 == 0 or kind != "ins":
            log(f"batch {i} {kind}: {u} updates in {dt * 1e3:.2f} ms, sweeps {sweeps[-1]}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.plds_set_timing(g.h, 0)
    value = tot["updates"] / wall
    log(f"timed: {tot['updates']} updates in {wall:.3f}s -> {value:.3e}/s")
    rc = g.check()
    lat_ms = sorted(x * 1e3 for x in lat)
    info = g.info()
    out = {
        "metric": METRIC, "value": value, "unit": "edge updates/s", "n_gpus": 1, "steps": len(plan), "warmup": 0,
        "ms_per_step": wall / len(plan) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16-streamed-ins{B}-then-2del-1mix", "n": n, "m0": m0, "delta": 0.4,
                   "lambda": 3.0, "batch": B, "K": info["K"],
                   "step": "one batch: the insertion stream of the whole graph, then deletions and a mixed batch"},
        "rates": {k: (v[0] / v[1] if v[1] else None) for k, v in per_kind.items()},
        "batch_latency_ms": {"p50": lat_ms[len(lat_ms) // 2], "p99": lat_ms[min(len(lat_ms) - 1,
                                                                              int(0.99 * len(lat_ms)))]},
        "sweeps_per_insert_batch": {"mean": float(np.mean(sweeps[:-3])), "max": int(np.max(sweeps[:-3]))},
        "roofline": roofline(tot, args.kernel),
        "device_check": rc,
        "slab_slots": info["slab_slots"],
    }
    print(json.dumps(out), flush=True)


def batched_workload(k, W, np):
    """The graphs and measured batches of the batched form (seed 4000 + i)."""
    return W.batched_graphs(k)


def tuning_batches(graphs, W):
    """One more batch per graph, of the measured batch's kind and size, drawn
    with other seeds (4700 + i): the schedule search runs on these, never on
    the measured batches."""
    out = []
    for i, (n, e, (kind, b)) in enumerate(graphs):
        size = len(b)
        out.append((kind, W.new_pairs(n, e, size, 4700 + i) if kind == "ins"
                    else W.sample_edges(e, min(size, len(e)), 4700 + i)))
    return out


def run_batched(args, P, W, torch, np):
    from paper_2106_03824_amd import autotune as AT
    k = args.graphs
    t = time.perf_counter()
    graphs = batched_workload(k, W, np)
    tunes = tuning_batches(graphs, W)
    ns = [n for n, _, _ in graphs]
    log(f"{k} graphs, {sum(ns)} vertices, {sum(len(e) for _, e, _ in graphs)} edges, "
        f"generated in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda", 0)
    gpu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    build = [gpu(e) for _, e, _ in graphs]
    kinds = [kd for _, _, (kd, _) in graphs]
    split = lambda bs: ([bs[g] if kinds[g] == "ins" else None for g in range(k)],
                        [bs[g] if kinds[g] == "del" else None for g in range(k)])
    ins_l, del_l = split([gpu(b) for _, _, (_, b) in graphs])
    tin_l, tdel_l = split([gpu(b) for _, b in tunes])
    mg = P.MultiPLDS(ns)
    singles = [P.PLDS(n) for n in ns]
    mg.update_multi(ins=build)
    for g in range(k):
        P.plds_update(singles[g].h, build[g], None)
    torch.cuda.synchronize()
    log("built")
    # the schedule search, on the tuning batches
    if args.tune_reps > 0:
        best, rec = AT.tune(mg, lambda: P.plds_update_multi(mg.h, tin_l, tdel_l), torch, reps=args.tune_reps,
                            log=log, path=args.tune_record, workload=f"batched-{k}-graphs tuning batches")
        log(f"tuned schedule {best}: {rec['best']['ms']:.2f} ms vs default {rec['default']['ms']:.2f} ms "
            f"({len(rec['trials'])} schedules timed)")
    else:
        best, rec = {}, {"trials": []}
    reps = max(args.steps, 1)
    e0, l0 = mg.dump()
    s_state = [sg.dump() for sg in singles]

    def fused(cfg):
        P.plds_set_launch(mg.h, **cfg)
        ts = []
        for r in range(reps + 1):
            mg.load(e0, l0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.plds_update_multi(mg.h, ins_l, del_l)
            torch.cuda.synchronize()
            if r:
                ts.append(time.perf_counter() - t0)
        st = mg.stats()
        return sorted(ts)[len(ts) // 2], st["applied_ins"] + st["applied_del"], st

    def loop():
        ts = []
        for r in range(reps + 1):
            for g in range(k):
                singles[g].load(*s_state[g])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, steps = 0, []
            for g in range(k):
                P.plds_update(singles[g].h, ins_l[g], del_l[g])
                st = singles[g].stats()
                u += st["applied_ins"] + st["applied_del"]
                steps.append(st["sweeps_ins"] + st["sweeps_del"])
            torch.cuda.synchronize()
            if r:
                ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2], u, steps

    t_def, u_def, _ = fused({})
    lv_def = mg.levels()
    t_fused, u_fused, s = fused(best)
    lv = mg.levels()
    t_loop, u_loop, loop_steps = loop()
    same = torch.equal(lv, lv_def) and all(torch.equal(mg.graph_levels(g, lv), singles[g].levels())
                                           for g in range(k))
    log(f"loop {u_loop} updates in {t_loop * 1e3:.1f} ms, batched {u_fused} in {t_fused * 1e3:.1f} ms "
        f"(default schedule {t_def * 1e3:.1f} ms), identical levels: {same}")
    out = {
        "metric": METRIC, "value": u_fused / t_fused, "unit": "edge updates/s", "n_gpus": 1, "steps": reps,
        "warmup": 1, "ms_per_step": t_fused * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batched-{k}-graphs-er-rmat-n2^10..2^16", "graphs": k, "vertices": sum(ns),
                   "delta": 0.4, "lambda": 3.0,
                   "step": "one measured batch per graph, all graphs in one call, from the post-build state"},
        "per_graph_loop": {"value": u_loop / t_loop, "ms": t_loop * 1e3},
        "default_schedule": {"value": u_def / t_def, "ms": t_def * 1e3},
        "schedule": best, "schedules_timed": len(rec["trials"]),
        "speedup_vs_loop": t_loop / t_fused,
        "identical_levels": same, "updates": u_fused, "level_steps": s["sweeps_ins"] + s["sweeps_del"],
        "insertion_steps": {"all": s["ins_steps"], "single_block_loop": s["ins_loop_steps"],
                            "loop_launches": s["ins_loop_launches"]},
        "level_steps_alone": {"max": max(loop_steps), "sum": sum(loop_steps)},
    }
    return out


def run_vertex(args, P, W, torch, np):
    """Vertex updates on the RMAT-20 graph of the default run (after its build):
    batches of 1e4 uniform random vertex deletions (each a batch of its edges'
    deletions), then a rebuild that renumbers the vertices left with edges
    consecutively.  `value` is deleted edges per second over the timed
    vertex-deletion batches.  The roofline is the deletion list's
    application (the largest kernel of a vertex batch): 56 bytes per applied
    deletion (the pair, both endpoints' slab tombstones, levels and
    counters)."""
    scale = 20
    m0 = 16 * 2 ** scale
    dev = torch.device("cuda", 0)
    st = W.RmatStream(scale, m0, seed=1, build_batches=16, cfg=2)
    n = st.n
    g = P.PLDS(n, 0.4, 3.0, 0, 2 * m0)
    for b in st.build:
        P.plds_batch_insert(g.h, torch.from_numpy(np.ascontiguousarray(b)).to(dev))
    rng = np.random.default_rng(4100)
    batches = [torch.from_numpy(rng.integers(0, n, 10 ** 4).astype(np.int32)).to(dev)
               for _ in range(args.warmup + args.steps)]
    torch.cuda.synchronize()
    edges, secs = 0, 0.0
    t_launches, t_ms, t_applied = 0, 0.0, 0
    for i, vs in enumerate(batches):
        if i == args.warmup:
            P.plds_set_timing(g.h, "apply_del")
        m_before = g.info()["m"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.plds_delete_vertices(g.h, vs)
        dt = time.perf_counter() - t0
        k = m_before - g.info()["m"]
        log(f"vertex batch {i}: 1e4 vertices, {k} edges deleted in {dt * 1e3:.2f} ms")
        if i >= args.warmup:
            edges += k
            secs += dt
            s = g.stats()
            t_launches += s["timed_launches"]
            t_ms += s["timed_ms"]
            t_applied += s["applied_del"]
    P.plds_set_timing(g.h, 0)
    roof = None
    if t_launches and t_ms > 0:
        per = 56 * t_applied / t_launches
        ach = per / (t_ms / t_launches * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_apply_del",
                "avg_launch_us": round(t_ms / t_launches * 1e3, 3), "launches": t_launches,
                "alg_bytes_per_launch": round(per, 1)}
    deg = g.degrees()
    keep = deg > 0
    relabel = torch.full((n,), -1, dtype=torch.int32, device=dev)
    n2 = int(keep.sum().item())
    relabel[keep] = torch.arange(n2, dtype=torch.int32, device=dev)
    m_now = g.info()["m"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g2 = g.rebuild(n2, relabel)
    torch.cuda.synchronize()
    t_rb = time.perf_counter() - t0
    ok = g2.check() == 0 and g2.info()["m"] == m_now
    log(f"rebuild: {n2} vertices, {m_now} edges in {t_rb * 1e3:.1f} ms, invariants {ok}")
    out = {
        "metric": "vertex deletions: deleted edges/s", "value": edges / secs, "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16-delete-1e4-vertices-then-rebuild", "n": n, "delta": 0.4,
                   "lambda": 3.0},
        "rebuild": {"vertices": n2, "edges": m_now, "ms": t_rb * 1e3, "edges_per_s": m_now / t_rb,
                    "invariants_hold": ok},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_vertex(st_edges_after_build(st), n, [b.cpu().numpy() for b in batches],
                                                  args.warmup)
    print(json.dumps(out), flush=True)


def run_static(args, P, W, torch, np):
    """Algorithm 6 on the RMAT-20 graph of the default run (after its 16
    build batches): `value` is edges per second of one static run at the
    first eps; the others are reported beside it.  The roofline is the relax
    kernel's over the timed runs at the first eps: per adjacency slot 4 bytes
    of neighbour id and 4 of its bucket (2m slots per run), per count update
    of an alive neighbour 8 bytes."""
    scale = 20
    m0 = 16 * 2 ** scale
    dev = torch.device("cuda", 0)
    st = W.RmatStream(scale, m0, seed=1, build_batches=16, cfg=2)
    n = st.n
    g = P.PLDS(n, 0.4, 3.0, 0, 2 * m0)
    for b in st.build:
        P.plds_batch_insert(g.h, torch.from_numpy(np.ascontiguousarray(b)).to(dev))
    m = g.info()["m"]
    out_t = torch.empty(n, dtype=torch.float64, device=dev)
    res = {}
    roof = None
    for eps in args.static_eps:
        for _ in range(args.warmup):
            P.plds_static_kcore(g.h, eps, out_t)
        # the relax kernel is timed in the runs at the first eps (the value's)
        first = eps == args.static_eps[0]
        if first:
            P.plds_set_timing(g.h, "sk_relax")
        s0 = g.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P.plds_static_kcore(g.h, eps, out_t)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        s = g.stats()
        if first:
            P.plds_set_timing(g.h, 0)
            launches = s["timed_launches"] - s0["timed_launches"]
            ms = s["timed_ms"] - s0["timed_ms"]
            alg = s["alg_bytes_peel"] - s0["alg_bytes_peel"]
            if launches > 0 and ms > 0:
                per = alg / launches
                ach = per / (ms / launches * 1e-3) / 1e9
                roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_sk_relax",
                        "avg_launch_us": round(ms / launches * 1e3, 3), "launches": launches,
                        "alg_bytes_per_launch": round(per, 1)}
        est = out_t.cpu().numpy()
        res[eps] = {"ms": dt * 1e3, "edges_per_s": m / dt, "host_syncs": s["host_syncs"],
                    "distinct_estimates": int(np.unique(est).size), "max_estimate": float(est.max())}
        log(f"static eps={eps}: {dt * 1e3:.2f} ms, {m / dt:.3e} edges/s")
    e0 = args.static_eps[0]
    out = {
        "metric": "static approximate k-core (Algorithm 6): edges/s", "value": res[e0]["edges_per_s"],
        "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res[e0]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16-static-kcore", "n": n, "m": m, "eps": e0},
        "per_eps": {str(k): v for k, v in res.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_static(e0)
    print(json.dumps(out), flush=True)


def run_orient(args, P, W, torch, np):
    """The RMAT-20 stream of the default run with orientation tracking on:
    every 1e6 batch (insertions, deletions, mixed) is followed by its flips F
    and oriented updates J (Algorithm 5).  Each batch is timed from before the
    update to after both outputs are in HBM; `value` counts the batch's
    applied updates over those times.  The roofline is the flip scan's: per
    searched edge 4 bytes of neighbour id and 8 of its two levels, per moved
    vertex 8 bytes of its own levels, per flip 8 bytes out."""
    scale, B = 20, args.batch
    m0 = 16 * 2 ** scale
    dev = torch.device("cuda", 0)
    st = W.RmatStream(scale, m0, seed=1, build_batches=16, cfg=2)
    n = st.n
    g = P.PLDS(n, 0.4, 3.0, 0, 2 * m0)
    for b in st.build:
        P.plds_batch_insert(g.h, torch.from_numpy(np.ascontiguousarray(b)).to(dev))
    P.plds_track_orientation(g.h, True)
    rounds = args.warmup + args.steps
    batches = []
    for r in range(rounds):
        ins = st.insert_batch(B)
        dele = st.delete_batch(B)
        mi, md = st.mixed_batch(B)
        batches += [("ins", torch.from_numpy(ins).to(dev), None), ("del", None, torch.from_numpy(dele).to(dev)),
                    ("mix", torch.from_numpy(mi).to(dev), torch.from_numpy(md).to(dev))]
    fcap = 16 * B
    fout = torch.empty((fcap, 2), dtype=torch.int32, device=dev)
    ji = torch.empty((B, 2), dtype=torch.int32, device=dev)
    jd = torch.empty((B, 2), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    log("orient: built, batches ready")
    tot = {"updates": 0, "seconds": 0.0, "flips": 0, "moved": 0, "searched": 0, "timed_ms": 0.0, "launches": 0,
           "out_s": 0.0}
    prev = g.levels().clone()
    for i, (kind, ins, dele) in enumerate(batches):
        timed = i >= 3 * args.warmup
        if timed and i == 3 * args.warmup:
            P.plds_set_timing(g.h, "flip_scan")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.plds_update(g.h, ins, dele)
        s = g.stats()
        t1 = time.perf_counter()
        k = P.plds_flips(g.h, fout)
        ni, nd = P.plds_oriented_updates(g.h, ji, jd)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s2 = g.stats()
        cur = g.levels()
        moved = cur != prev
        deg = g.degrees()
        nm = int(moved.sum().item())
        srch = int(deg[moved].sum().item())
        prev = cur.clone()
        if k > fcap:
            raise RuntimeError(f"{k} flips exceed the buffer of {fcap}")
        u = s["applied_ins"] + s["applied_del"]
        assert (ni, nd) == (s["applied_ins"], s["applied_del"])
        log(f"batch {i} {kind}: {u} updates, {k} flips, {nm} moved vertices, {srch} searched edges, "
            f"update {1e3 * (t1 - t0):.2f} ms + F,J {1e3 * (t2 - t1):.2f} ms")
        if timed:
            tot["updates"] += u
            tot["seconds"] += t2 - t0
            tot["out_s"] += t2 - t1
            tot["flips"] += k
            tot["moved"] += nm
            tot["searched"] += srch
            tot["timed_ms"] += s2["timed_ms"]
            tot["launches"] += s2["timed_launches"]
    P.plds_set_timing(g.h, 0)
    nb = 3 * args.steps
    alg = 12 * tot["searched"] + 8 * tot["moved"] + 8 * tot["flips"]
    roof = None
    if tot["launches"] and tot["timed_ms"] > 0:
        avg_ms = tot["timed_ms"] / tot["launches"]
        per = alg / tot["launches"]
        ach = per / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_flip_scan",
                "avg_launch_us": round(avg_ms * 1e3, 3), "launches": tot["launches"],
                "alg_bytes_per_launch": round(per, 1)}
    out = {
        "metric": "edge updates/s with orientation outputs (F, J) at 1e6 batch",
        "value": tot["updates"] / tot["seconds"], "unit": "edge updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tot["seconds"] / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16-build16-then-ins/del/mix-{B}-with-flips", "n": n, "m0": m0,
                   "delta": 0.4, "lambda": 3.0, "batch": B,
                   "step": "1 insertion + 1 deletion + 1 mixed batch, each followed by F and J"},
        "flips_per_batch": tot["flips"] / nb, "moved_per_batch": tot["moved"] / nb,
        "searched_edges_per_batch": tot["searched"] / nb, "orientation_ms_per_batch": tot["out_s"] / nb * 1e3,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_orient()
    print(json.dumps(out), flush=True)


def run_serve(args, P, W, torch, np):
    """Resident R-MAT graphs behind the continuous-batching
    server (shards of multi-graph handles; the pending requests of a shard's
    graphs are served by one fused update call and one coreness call).
    Request streams at saturation and at fractions of it; then the same
    graphs and requests served one at a time with a plain handle per graph
    (the per-graph plain launches), whose results must be identical."""
    import random
    from paper_2106_03824_amd import serve as S

    def fresh(reqs):   # unserved copies sharing the (read-only) payloads
        return [S.Request(r.rid, r.graph, r.kind, r.arrival, r.payload) for r in reqs]

    rng = random.Random(5000)
    lo, hi = args.serve_scales
    t = time.perf_counter()
    graphs = {}
    for g in range(args.serve_graphs):
        sc = rng.randint(lo, hi)
        graphs[g] = (2 ** sc, W.rmat(sc, 16 * 2 ** sc, seed=5000 + g))
    m_total = sum(len(e) for _, e in graphs.values())
    log(f"{len(graphs)} graphs, {m_total} edges, generated in {time.perf_counter() - t:.1f}s")
    N = args.serve_requests
    admits = [S.Request(g, g, "admit", 0.0, graphs[g]) for g in graphs]
    retires = [S.Request(10 ** 9 + g, g, "retire", 0.0) for g in graphs]
    srv = S.Server(1 << 60, slots=args.slots)
    t_build = srv.serve(fresh(admits), arrival=False)
    log(f"admitted and built in {t_build:.1f}s ({len(srv.shards)} shards of {args.slots} slots)")
    applied = lambda tr: sum(r.result["applied_ins"] + r.result["applied_del"] for r in tr
                             if r.kind == "update" and r.result)
    served, runs = [], []
    sat_rps = None
    for k, f in enumerate((None, 0.1, 0.5, 0.9, 1.2)):
        tr = S.make_updates(graphs, N, None if f is None else f * sat_rps, 5100 + k, rid0=(k + 1) * 10 ** 6)
        served.append(tr)
        c0, r0 = srv.fused_calls, srv.fused_requests
        wall = srv.serve(tr, arrival=f is not None)
        if f is None:
            sat_rps = N / wall
        runs.append({"rate_factor": f, "offered_per_s": None if f is None else f * sat_rps,
                     "requests_per_s": N / wall, "updates_per_s": applied(tr) / wall,
                     "requests_per_fused_call": (srv.fused_requests - r0) / max(srv.fused_calls - c0, 1),
                     **S.latency_stats(tr)})
        log(f"rate {'saturation' if f is None else f}: {N / wall:.1f} requests/s, "
            f"{applied(tr) / wall:.3e} updates/s, p50 {runs[-1]['p50_ms']:.2f} ms, p99 {runs[-1]['p99_ms']:.2f} ms, "
            f"{runs[-1]['requests_per_fused_call']:.1f} requests per fused call")
    mixed_ret = fresh(retires)
    srv.serve(mixed_ret, arrival=False)
    srv.close()
    # the same graphs and requests, one request at a time, a plain handle per graph
    alone_all = fresh(admits) + [r for tr in served for r in fresh(tr)] + fresh(retires)
    t = time.perf_counter()
    S.serve_alone(alone_all, progress=lambda i: log(f"one at a time: {i} of {len(alone_all)} requests"))
    log(f"one at a time: {time.perf_counter() - t:.1f}s")
    by_rid = {r.rid: r for r in alone_all}
    sat_alone = served[0]
    t_alone = sum(by_rid[r.rid].done - by_rid[r.rid].start for r in sat_alone)
    same, errors = True, 0
    for tr in served:
        for x in tr:
            y = by_rid[x.rid]
            errors += (x.error is not None) + (y.error is not None)
            if x.kind == "query":
                same = same and np.array_equal(x.result.view(np.int64), y.result.view(np.int64))
            elif x.kind == "update":
                same = same and x.result == y.result
    for x in mixed_ret:
        same = same and np.array_equal(x.result["levels"], by_rid[x.rid].result["levels"])
    log(f"identical to one-at-a-time serving: {same}, errors {errors}")
    out = {
        "metric": METRIC, "value": runs[0]["updates_per_s"], "unit": "edge updates/s", "n_gpus": 1,
        "steps": N, "warmup": 0, "ms_per_step": 1e3 / sat_rps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"serving-{len(graphs)}-rmat-scale{lo}..{hi}-ef16", "graphs": len(graphs),
                   "edges": m_total, "slots_per_shard": args.slots, "requests_per_run": N,
                   "step": "one request: an update batch (1e2..1e6, 70% ins) or a 1e3-vertex coreness query"},
        "latency": runs, "identical_to_alone": same, "errors": errors, "build_s": t_build,
        "one_at_a_time": {"updates_per_s": applied([by_rid[r.rid] for r in sat_alone]) / t_alone,
                          "seconds": t_alone,
                          "note": "the saturation run's requests served one at a time with a plain handle per "
                                  "graph (sum of their service times)"},
    }
    return out


def st_edges_after_build(st):
    """Edge set right after the build (the stream tracks later batches)."""
    import numpy as np
    return np.concatenate(st.build)


if __name__ == "__main__":
    main()
