"""Launch-schedule search for the level loops.

How many workgroups the sweep kernels get, and how many insertion steps go
into one prebuilt HIP graph (``plds_set_launch``), change how fast a batch
runs and never what it computes.  ``tune`` times candidate schedules on a
caller's workload and keeps the fastest:

* the handle's state is dumped once (``plds_dump_state``) and loaded back
  (``plds_load_state``) before every trial, so each trial applies the same
  workload to the same state;
* every schedule first gets one untimed trial (it builds that schedule's
  step graphs), then ``reps`` timed ones; its time is their median;
* the levels a trial ends with must equal those of the very first trial,
  bit for bit, or the search stops with an error -- a schedule that changed
  a result would be a bug, not a speed-up;
* the search is a coordinate descent from the default schedule: each field
  in turn takes every value of its candidate list with the other fields
  fixed, the fastest value stays, and passes repeat until one changes
  nothing (at most ``passes``).

The record lists every timed schedule, the default's time and the winner's,
and can be written as JSON.  The handle is left holding the winning schedule
and the dumped state.
"""
import json
import statistics
import time

from . import plds as P

# candidate values per field (plds_launch_t); the defaults are among them
SPACE = {
    "scan_blocks": (256, 512, 768, 1024, 1280, 1536, 1792, 2048),
    "graph_steps": (4, 8, 16, 32),
    "dl_blocks": (256, 512, 1024, 2048),
    "del_scan_blocks": (512, 1024, 2048, 4096),
}


def _key(cfg):
    return tuple(cfg[f] for f in P.LAUNCH_FIELDS)


def tune(h, run, torch, space=None, reps=3, passes=2, log=None, path=None, workload=""):
    """Searches launch schedules for handle ``h`` (a ``PLDS``/``MultiPLDS``
    or its raw pointer) on the workload ``run()``, a callable that applies
    update calls to that handle.  Returns ``(best, record)``: the winning
    schedule (a dict of ``plds_launch_t`` fields) and the search record.
    ``path``: where to write the record as JSON (optional)."""
    space = dict(SPACE if space is None else space)
    hp = getattr(h, "h", h)
    say = log or (lambda *_: None)
    m = P.plds_info(hp)["m"]
    n = P.plds_info(hp)["n"]
    edges = torch.empty((max(m, 1), 2), dtype=torch.int32, device="cuda")
    levels0 = torch.empty(n, dtype=torch.int32, device="cuda")
    got = P.plds_dump_state(hp, edges, levels0)
    edges = edges[:got]
    ref = None
    timed = {}
    trials = []

    def trial(cfg):
        nonlocal ref
        k = _key(cfg)
        if k in timed:
            return timed[k]
        P.plds_set_launch(hp, **cfg)
        ts = []
        for r in range(reps + 1):
            P.plds_load_state(hp, edges, levels0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lv = torch.empty(n, dtype=torch.int32, device="cuda")
            P.plds_levels(hp, lv)
            if ref is None:
                ref = lv
            elif not torch.equal(lv, ref):
                raise RuntimeError(f"schedule {cfg} changed the levels")
            if r:   # the first run builds the schedule's step graphs
                ts.append(dt)
        ms = statistics.median(ts) * 1e3
        timed[k] = ms
        trials.append({"schedule": dict(cfg), "ms": ms, "runs_ms": [t * 1e3 for t in ts]})
        say(f"schedule {cfg}: {ms:.3f} ms")
        return ms

    P.plds_set_launch(hp)   # all defaults
    default = P.plds_get_launch(hp)
    best = dict(default)
    best_ms = trial(best)
    default_ms = best_ms
    done_passes = 0
    for _ in range(passes):
        done_passes += 1
        changed = False
        for f in P.LAUNCH_FIELDS:
            for v in space.get(f, ()):
                cfg = dict(best, **{f: int(v)})
                ms = trial(cfg)
                if ms < best_ms:
                    best, best_ms, changed = cfg, ms, True
        if not changed:
            break
    P.plds_set_launch(hp, **best)
    P.plds_load_state(hp, edges, levels0)
    torch.cuda.synchronize()
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    record = {
        "workload": workload, "device": dev.name, "reps": reps, "passes": done_passes,
        "space": {f: list(space.get(f, ())) for f in P.LAUNCH_FIELDS},
        "default": {"schedule": default, "ms": default_ms},
        "best": {"schedule": best, "ms": best_ms},
        "speedup_vs_default": default_ms / best_ms if best_ms > 0 else None,
        "trials": trials,
    }
    if path:
        with open(path, "w") as f:
            json.dump(record, f, indent=1)
    return best, record
