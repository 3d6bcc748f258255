"""Serving loop: many resident dynamic graphs on the GPU, fed by a stream of
requests (admit a graph, apply an update batch, answer a coreness query,
retire a graph), with continuous batching.

Resident graphs live in shards.  A shard is one multi-graph handle
(plds_create_multi) with a fixed number of graph slots of one size class
(a power of two of vertices); a graph is admitted into a free slot of its
class (plds_reset_graph gives the slot the graph's own n, levels per group
and thresholds, so the graph goes through the states of a handle of its
own).  Every shard has a worker thread with its own HIP stream, so the
shards' work overlaps on the device.

Continuous batching.  A shard's worker repeatedly takes, for every graph of
the shard that has work, the request at the head of its queue (the oldest
first), and serves all of them together:

* the update batches of all those graphs, and the initial edges of the
  graphs being admitted, go into ONE fused plds_update_multi call (each
  graph gets Update(B) of Algorithm 1 with its own lists; graphs without a
  request are untouched);
* the coreness queries of all those graphs are answered by one
  plds_coreness call over their global vertex ids;
* retired graphs hand back their levels and free their slots.

Requests that arrive while a fused call runs join the next one.  A graph
takes at most one request per fused call, so its requests are applied one
at a time in arrival order, and every result is the one that serving the
graph alone, request by request, gives (tests/test_gpu_serve.py checks it,
and against the CPU oracle's replay).

Admission control: a graph is admitted only when its estimated HBM
footprint fits in the remaining budget; until then its requests wait, and
retiring a graph frees its footprint.  A shard is created when a graph
needs a slot of a class that has none free.  An admission that fails (the
library refused to create the shard, or a request carried ids outside the
graph's range) fails that request; the later requests of a graph whose
admission failed fail at once with the same error, so the loop drains.
A fused call that fails as a whole (out of device memory) fails every
request in it.

The server does no arithmetic of the method; it only orders calls into the
library (plds.py / libplds.so).
"""
import collections
import heapq
import threading
import time

import numpy as np

from . import plds as P


def footprint_bytes(n, m, batch=10 ** 6):
    """HBM estimate of one graph: the per-vertex arrays (about 26 int32 and
    3 int64 per vertex), the adjacency pool (2m slots at 60% load, plus the
    per-vertex floor the library reserves) and the batch scratch (hash set
    and edge lists)."""
    per_vertex = 26 * 4 + 3 * 8
    pool = max(1 << 20, 12 * n + (2 * m * 5) // 3) * 4
    scratch = 4 * batch * 8 + 2 * batch * 4
    return n * per_vertex + pool + scratch


def size_class(n, smallest=1024):
    c = smallest
    while c < n:
        c *= 2
    return c


class Request:
    """kind: 'admit' (n, edges), 'update' (ins, dele), 'query' (vertices),
    'retire'.  Arrays are host numpy int32 arrays (edges [k, 2]); the server
    moves them to the device on the shard's stream."""
    __slots__ = ("rid", "graph", "kind", "arrival", "payload", "start", "done", "result", "error", "fused")

    def __init__(self, rid, graph, kind, arrival, payload=None):
        self.rid, self.graph, self.kind, self.arrival, self.payload = rid, graph, kind, arrival, payload
        self.start = self.done = None
        self.result = None
        self.error = None
        self.fused = 0        # requests served by the same fused call


class Shard:
    def __init__(self, server, cls, slots):
        import torch
        self.cls, self.slots = cls, slots
        self.h = P.MultiPLDS([cls] * slots, server.delta, server.lam)
        self.free = list(range(slots))
        self.graph_of = {}                   # slot -> graph
        self.stream = torch.cuda.Stream()
        self.thread = threading.Thread(target=server._worker, args=(self,), daemon=True)


class Server:
    def __init__(self, budget_bytes, slots=8, delta=0.4, lam=3.0, fuse=True):
        """slots: graph slots per shard; fuse=False serves one request per
        library call (the one-at-a-time reference)."""
        import torch
        self.torch = torch
        self.budget = budget_bytes
        self.used = 0
        self.delta, self.lam = delta, lam
        self.slots = slots
        self.fuse = fuse
        self.shards = []
        self.where = {}                                     # graph -> (shard, slot)
        self.foot = {}                                      # graph -> admitted footprint
        self.failed = {}                                    # graph -> error of its failed admission
        self.queues = collections.defaultdict(collections.deque)
        self.busy = set()
        self.cv = threading.Condition()
        self.closed = False
        self.inflight = 0
        self.fused_calls = 0
        self.fused_requests = 0

    # ------------------------------------------------------------ intake
    def submit(self, req):
        with self.cv:
            if req.graph in self.failed and req.kind != "admit":
                self._fail(req, self.failed[req.graph])
                return
            self.queues[req.graph].append(req)
            if req.kind == "admit":
                err = self._grow(size_class(req.payload[0]))
                if err is not None:       # no slot can be made for it: this admission fails
                    self.queues[req.graph].pop()
                    self._fail(req, err)
                    self.failed[req.graph] = err
            self.cv.notify_all()

    def _fail(self, req, err):
        """Under the lock: complete a request that cannot run with an error."""
        req.start = req.done = time.perf_counter()
        req.error = err if req.kind == "admit" else RuntimeError(f"graph {req.graph} was not admitted: {err!r}")

    def _fail_graph(self, g, err):
        """Under the lock: graph g's admission failed; its queued requests
        fail at once, and so will later ones."""
        self.failed[g] = err
        q = self.queues.get(g)
        while q and q[0].kind != "admit":
            self._fail(q.popleft(), err)

    def _grow(self, cls):
        """Under the lock: a new shard of class `cls` while the admissions
        waiting for that class outnumber its free slots; the library's error
        if it cannot create one."""
        want = sum(1 for q in self.queues.values() for r in q if r.kind == "admit" and size_class(r.payload[0]) == cls)
        free = sum(len(s.free) for s in self.shards if s.cls == cls)
        while want > free:
            try:
                sh = Shard(self, cls, self.slots)
            except Exception as e:
                return e
            self.shards.append(sh)
            sh.thread.start()
            free += sh.slots
        return None

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for sh in self.shards:
            sh.thread.join()
        for sh in self.shards:
            sh.h.close()
        self.shards = []

    def drain(self):
        """Wait until every submitted request has finished."""
        with self.cv:
            while self.inflight or any(self.queues.values()):
                self.cv.wait(0.05)

    # ---------------------------------------------------------- schedule
    def _collect(self, sh):
        """Under the lock: the head request of every graph of shard `sh` (and
        of admissions it can place) that may start now, oldest first; at most
        one per graph (one when fusing is off).  Admissions take free slots
        and budget in arrival order."""
        heads = []
        for g, q in self.queues.items():
            if not q or g in self.busy:
                continue
            head = q[0]
            if head.kind == "admit":
                if size_class(head.payload[0]) == sh.cls:
                    heads.append(head)
            elif g in self.where and self.where[g][0] is sh:
                heads.append(head)
        heads.sort(key=lambda r: (r.arrival, r.rid))
        cands, avail, used = [], len(sh.free), self.used
        for r in heads:
            if r.kind == "admit":
                n, edges = r.payload
                need = footprint_bytes(n, len(edges))
                if avail == 0 or not (used + need <= self.budget or (not self.where and not self.busy and not cands)):
                    continue
                avail -= 1
                used += need
            cands.append(r)
            if not self.fuse:
                break
        for r in cands:
            self.queues[r.graph].popleft()
            self.busy.add(r.graph)
            self.inflight += 1
            if r.kind == "admit":
                self.failed.pop(r.graph, None)
                n, edges = r.payload
                slot = sh.free.pop(0)
                sh.graph_of[slot] = r.graph
                self.where[r.graph] = (sh, slot)
                f = footprint_bytes(n, len(edges))
                self.used += f
                self.foot[r.graph] = f
        return cands

    def _worker(self, sh):
        while True:
            with self.cv:
                batch = self._collect(sh)
                while not batch:
                    if self.closed:
                        return
                    self.cv.wait(0.05)
                    batch = self._collect(sh)
            t = time.perf_counter()
            for r in batch:
                r.start = t
                r.fused = len(batch)
            try:
                with self.torch.cuda.stream(sh.stream):
                    self._run(sh, batch)
                sh.stream.synchronize()
            except Exception as e:      # the fused call failed as a whole
                for r in batch:
                    if r.error is None and r.done is None:
                        r.error = e
            t = time.perf_counter()
            with self.cv:
                self.fused_calls += 1
                self.fused_requests += len(batch)
                for r in batch:
                    r.done = r.done or t
                    self.busy.discard(r.graph)
                    self.inflight -= 1
                    if r.kind == "admit" and r.error is not None:
                        self._release(r.graph)
                        self._fail_graph(r.graph, r.error)
                    elif r.kind == "retire" and r.error is None:
                        self._release(r.graph)
                self.cv.notify_all()

    def _release(self, g):
        """Under the lock: free graph g's slot and footprint."""
        if g in self.where:
            sh, slot = self.where.pop(g)
            sh.graph_of.pop(slot, None)
            sh.free.append(slot)
            sh.free.sort()
        self.used -= self.foot.pop(g, 0)

    def _dev(self, a):
        if a is None or len(a) == 0:
            return None
        return self.torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")

    @staticmethod
    def _ids_ok(a, n):
        return a is None or len(a) == 0 or (np.asarray(a).min() >= 0 and np.asarray(a).max() < n)

    def _run(self, sh, batch):
        torch = self.torch
        h = sh.h
        ins, dele = [None] * sh.slots, [None] * sh.slots
        upd = []
        for r in batch:
            if r.kind == "admit":
                n, edges = r.payload
                if not self._ids_ok(edges, n):
                    r.error = P.PLDSError(P.PLDS_ERANGE, "admit")
                    continue
                slot = self.where[r.graph][1]
                h.reset_graph(slot, n, stream=sh.stream)
                ins[slot] = self._dev(edges)
                upd.append((r, slot))
            elif r.kind == "update":
                a, b = r.payload
                slot = self.where[r.graph][1]
                n = h.ns[slot]
                if not (self._ids_ok(a, n) and self._ids_ok(b, n)):
                    r.error = P.PLDSError(P.PLDS_ERANGE, "update")
                    continue
                ins[slot], dele[slot] = self._dev(a), self._dev(b)
                upd.append((r, slot))
        if any(x is not None for x in ins) or any(x is not None for x in dele):
            P.plds_update_multi(h.h, ins, dele, stream=sh.stream)
            ai, ad = P.plds_graph_applied(h.h, sh.slots, stream=sh.stream)
        elif upd:
            ai = ad = [0] * sh.slots
        for r, slot in upd:
            r.result = ({"m": ai[slot], "applied_ins": ai[slot]} if r.kind == "admit" else
                        {"applied_ins": ai[slot], "applied_del": ad[slot]})
        # coreness queries of all graphs of the call, one library call
        qs = [r for r in batch if r.kind == "query" and r.error is None]
        if qs:
            gids = np.concatenate([np.asarray(r.payload, dtype=np.int64) + h.base[self.where[r.graph][1]]
                                   for r in qs]).astype(np.int32)
            bad = [not self._ids_ok(r.payload, h.ns[self.where[r.graph][1]]) for r in qs]
            vs = torch.from_numpy(gids).to("cuda")
            out = torch.empty(len(gids), dtype=torch.float64, device="cuda")
            P.plds_coreness(h.h, vs, out, stream=sh.stream)
            res = out.cpu().numpy()
            at = 0
            for r, b in zip(qs, bad):
                k = len(r.payload)
                if b:
                    r.error = P.PLDSError(P.PLDS_ERANGE, "query")
                else:
                    r.result = res[at:at + k].copy()
                at += k
        rets = [r for r in batch if r.kind == "retire" and r.error is None]
        if rets:
            lv = h.levels().cpu().numpy()
            for r in rets:
                slot = self.where[r.graph][1]
                r.result = {"levels": lv[h.base[slot]:h.base[slot] + h.ns[slot]].copy()}

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


def replay(requests, budget_bytes, slots=8, arrival=True, fuse=True):
    """Serve `requests` on a fresh server and close it; returns the wall time."""
    srv = Server(budget_bytes, slots, fuse=fuse)
    try:
        return srv.serve(requests, arrival)
    finally:
        srv.close()


def serve_alone(requests, delta=0.4, lam=3.0, progress=None):
    """The reference: every request on its own, in order of request id, each
    graph in a plain handle of its own (one library call per request).
    progress(i) is called every 100 requests."""
    import torch
    handles, out = {}, {}
    for i, r in enumerate(sorted(requests, key=lambda r: r.rid)):
        if progress is not None and i % 100 == 0:
            progress(i)
        t = time.perf_counter()
        r.start = t
        try:
            if r.kind == "admit":
                n, edges = r.payload
                h = P.PLDS(n, delta, lam, 0, len(edges))
                handles[r.graph] = h
                if len(edges):
                    h.update(edges, None)
                s = h.stats()
                r.result = {"m": h.info()["m"], "applied_ins": s["applied_ins"]}
            elif r.kind == "update":
                h = handles[r.graph]
                h.update(*r.payload)
                s = h.stats()
                r.result = {"applied_ins": s["applied_ins"], "applied_del": s["applied_del"]}
            elif r.kind == "query":
                h = handles[r.graph]
                vs = torch.as_tensor(np.asarray(r.payload, dtype=np.int32)).to("cuda")
                r.result = h.coreness(vs).cpu().numpy()
            elif r.kind == "retire":
                h = handles.pop(r.graph)
                r.result = {"levels": h.levels().cpu().numpy()}
                h.close()
        except Exception as e:
            r.error = e
        torch.cuda.synchronize()
        r.done = time.perf_counter()
    for h in handles.values():
        h.close()
    return out


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
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    fused = np.array([r.fused for r in reqs])
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "mean_fused": float(fused.mean()) if len(fused) else 0.0}
