"""Serving loop: many resident dynamic graphs, each a PLDS handle on the GPU,
fed by a stream of requests (admit a graph, apply an update batch, answer a
coreness query, retire a graph).

Scheduling is continuous and work-conserving.  A pool of worker threads,
each with its own HIP stream, runs requests as soon as they may run.  The
GIL is released inside the library calls, so work of different graphs
overlaps on the device.  Two rules keep every result identical to serving
each graph alone, in arrival order:

* the requests of one graph run one at a time, in arrival order (a graph
  is busy while one of its requests runs);
* among the graphs that are not busy, the oldest waiting request runs first.

Admission control: a graph is admitted only when its estimated HBM
footprint fits in the remaining budget.  Until then its requests wait.
Retiring a graph frees its footprint and lets waiting graphs in.  An
admission that fails (the library refused to create the handle or to load
the initial edges) frees the footprint and leaves nothing resident; every
later request of that graph fails at once with the same error.

The server does no arithmetic of the method; it only orders calls into the
library (plds.py / libplds.so).
"""
import collections
import heapq
import threading
import time

from . import plds as P


def footprint_bytes(n, m, batch=10 ** 6):
    """HBM estimate of one handle: the per-vertex arrays (about 26 int32 and
    3 int64 per vertex), the adjacency pool (2m slots at 60% load, plus the
    per-vertex floor the library reserves) and the batch scratch (hash set
    and edge lists)."""
    per_vertex = 26 * 4 + 3 * 8
    pool = max(1 << 20, 12 * n + (2 * m * 5) // 3) * 4
    scratch = 4 * batch * 8 + 2 * batch * 4
    return n * per_vertex + pool + scratch


class Request:
    """kind: 'admit' (n, edges), 'update' (ins, dele), 'query' (vertices),
    'retire'.  Arrays are host numpy int32 arrays (edges [k, 2]); the server
    moves them to the device on the worker's stream."""
    __slots__ = ("rid", "graph", "kind", "arrival", "payload", "start", "done", "result", "error")

    def __init__(self, rid, graph, kind, arrival, payload=None):
        self.rid, self.graph, self.kind, self.arrival, self.payload = rid, graph, kind, arrival, payload
        self.start = self.done = None
        self.result = None
        self.error = None


class Server:
    def __init__(self, budget_bytes, workers=8, delta=0.4, lam=3.0):
        import torch
        self.torch = torch
        self.budget = budget_bytes
        self.used = 0
        self.delta, self.lam = delta, lam
        self.handles = {}                                   # graph -> PLDS
        self.foot = {}                                      # graph -> admitted footprint
        self.failed = {}                                    # graph -> error of its failed admission
        self.queues = collections.defaultdict(collections.deque)
        self.busy = set()
        self.cv = threading.Condition()
        self.closed = False
        self.inflight = 0
        self.streams = [torch.cuda.Stream() for _ in range(workers)]
        self.threads = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(workers)]
        for t in self.threads:
            t.start()

    # ------------------------------------------------------------ intake
    def submit(self, req):
        with self.cv:
            self.queues[req.graph].append(req)
            self.cv.notify_all()

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        for g in list(self.handles):
            self.handles.pop(g).close()

    def drain(self):
        """Wait until every submitted request has finished."""
        with self.cv:
            while self.inflight or any(self.queues.values()):
                self.cv.wait(0.05)

    # ---------------------------------------------------------- schedule
    def _runnable(self, req):
        """Under the lock: may the head request of its graph start now?"""
        if req.kind == "admit":
            n, edges = req.payload
            need = footprint_bytes(n, len(edges))
            return self.used + need <= self.budget or not self.handles and not self.busy
        return req.graph in self.handles or req.graph in self.failed

    def _pick(self):
        best = None
        for g, q in self.queues.items():
            if not q or g in self.busy:
                continue
            head = q[0]
            if not self._runnable(head):
                continue
            if best is None or head.arrival < best.arrival:
                best = head
        if best is not None:
            self.queues[best.graph].popleft()
            self.busy.add(best.graph)
            self.inflight += 1
            if best.kind == "admit":
                n, edges = best.payload
                f = footprint_bytes(n, len(edges))
                self.used += f
                self.foot[best.graph] = f
        return best

    def _worker(self, i):
        torch = self.torch
        stream = self.streams[i]
        while True:
            with self.cv:
                req = self._pick()
                while req is None:
                    if self.closed:
                        return
                    self.cv.wait(0.05)
                    req = self._pick()
            req.start = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    self._run(req, stream)
                stream.synchronize()
            except Exception as e:      # reported per request
                req.error = e
            req.done = time.perf_counter()
            with self.cv:
                self.busy.discard(req.graph)
                self.inflight -= 1
                if req.kind == "retire" or (req.kind == "admit" and req.error is not None):
                    self.used -= self.foot.pop(req.graph, 0)
                if req.kind == "admit" and req.error is not None:
                    self.failed[req.graph] = req.error
                self.cv.notify_all()

    def _dev(self, a, stream):
        """Host array -> device tensor, copied on the worker's stream (the
        current stream inside _run)."""
        import numpy as np
        if a is None or len(a) == 0:
            return None
        return self.torch.from_numpy(np.ascontiguousarray(a)).to("cuda")

    def _run(self, req, stream):
        torch = self.torch
        if req.graph in self.failed and req.kind != "admit":
            raise RuntimeError(f"graph {req.graph} was not admitted: {self.failed[req.graph]!r}")
        if req.kind == "admit":
            n, edges = req.payload
            self.failed.pop(req.graph, None)
            h = P.PLDS(n, self.delta, self.lam, 0, len(edges))
            try:
                if len(edges):
                    P.plds_update(h.h, self._dev(edges, stream), None, stream=stream)
                req.result = {"m": h.info()["m"]}
            except Exception:
                h.close()
                raise
            self.handles[req.graph] = h
        elif req.kind == "update":
            ins, dele = req.payload
            h = self.handles[req.graph]
            P.plds_update(h.h, self._dev(ins, stream), self._dev(dele, stream), stream=stream)
            s = h.stats()
            req.result = {"applied_ins": s["applied_ins"], "applied_del": s["applied_del"]}
        elif req.kind == "query":
            h = self.handles[req.graph]
            vs = self._dev(req.payload, stream)
            out = torch.empty(len(req.payload), dtype=torch.float64, device="cuda")
            P.plds_coreness(h.h, vs, out, stream=stream)
            req.result = out.cpu().numpy()
        elif req.kind == "retire":
            h = self.handles.pop(req.graph)
            req.result = {"levels": h.levels().cpu().numpy()}
            h.close()
        else:
            raise ValueError(req.kind)


    def serve(self, requests, arrival=True):
        """Feed `requests` (their `arrival` in seconds from now) and wait
        until all are done; with arrival=False all arrive at once.  Each
        request's `arrival` becomes an absolute perf_counter time.  Returns
        the wall time."""
        t0 = time.perf_counter()
        heap = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(heap)
        while heap:
            at, _, r = heapq.heappop(heap)
            if arrival:
                wait = t0 + at - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                r.arrival = t0 + at
            else:
                r.arrival = t0
            self.submit(r)
        self.drain()
        return time.perf_counter() - t0


def replay(requests, budget_bytes, workers, arrival=True):
    """Serve `requests` on a fresh server and close it; returns the wall time."""
    srv = Server(budget_bytes, workers)
    try:
        return srv.serve(requests, arrival)
    finally:
        srv.close()


def make_updates(graphs, nreq, rate, seed, rid0=0, query_size=1000, size_range=(2, 6), ins_share=0.7):
    """A request stream over resident graphs {g: (n, initial edges)}: Poisson
    arrivals at `rate` per second; each request targets a uniform random
    graph and is, with probability 1/2, an update batch of log-uniform size
    in [10^size_range[0], 10^size_range[1]] (insertions of uniform random
    pairs with probability ins_share, else deletions sampled from the
    graph's initial edges; pairs already present or absent are no-ops by the
    batch semantics), or else a coreness query for `query_size` uniform
    random vertices.  rate=None: all at time 0."""
    import random
    import numpy as np
    from . import workloads as W
    rng = random.Random(seed)
    keys = sorted(graphs)
    reqs, t = [], 0.0
    for i in range(nreq):
        if rate:
            t += rng.expovariate(rate)
        g = keys[rng.randrange(len(keys))]
        n, e = graphs[g]
        r = np.random.default_rng([seed, i])
        if rng.random() < 0.5:
            size = int(round(10 ** rng.uniform(*size_range)))
            if rng.random() < ins_share:
                reqs.append(Request(rid0 + i, g, "update", t, (r.integers(0, n, size=(size, 2), dtype=np.int32),
                                                               None)))
            else:
                dele = W.sample_edges(e, min(size, len(e)), seed * 1000003 + i)
                reqs.append(Request(rid0 + i, g, "update", t, (None, dele)))
        else:
            reqs.append(Request(rid0 + i, g, "query", t, r.integers(0, n, size=query_size, dtype=np.int32)))
    return reqs


def latency_stats(reqs):
    import numpy as np
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}
