"""Independent pure-Python PLDS on tiny graphs, in exact rational arithmetic.

Used only to pin the C oracle.  It shares nothing with it: thresholds come
from ``fractions.Fraction``; every degree is recounted from the adjacency
sets; the insertion pass visits every level 0..K-1 and takes every vertex of
that level violating Invariant 1 (Algorithm 2); the deletion pass visits every
level 0..K-1 and moves every Invariant-2 violator whose desire-level equals
that level (Algorithm 3); the desire-level is taken literally from its
definition, by trying every level 0..K-1 and keeping the closest one at which
both invariants hold.

Options: a coefficient of Invariant 1 in place of 2 + 3/lambda (the
experiments' heuristic parameters use 1.1, taken as the exact rational of its
decimal text), and the implementation's insertion procedure (jump=True): at
every level 0..K-1 the vertices of that level violating Invariant 1 each take
their desire-level (the literal search above, made before any of them moves)
and all of them move there together.
"""
from fractions import Fraction
import math


def exact_params(n, delta, lam, levels_per_group=0, coeff=None):
    """t = least integer with (1+delta)^t >= n; L = 4t (or the override);
    G = t+1 groups; K = G*L levels (Section "Detailed PLDS Algorithm")."""
    delta, lam = Fraction(delta), Fraction(lam)
    t, p = 0, Fraction(1)
    while p < n:
        p *= 1 + delta
        t += 1
    L = levels_per_group if levels_per_group > 0 else max(1, 4 * t)
    G = t + 1
    coeff = 2 + 3 / lam if coeff is None else Fraction(str(coeff))
    up_max = [math.floor(coeff * (1 + delta) ** g) for g in range(G)]
    dn_min = [math.ceil((1 + delta) ** g) for g in range(G)]
    return dict(t=t, L=L, G=G, K=G * L, up_max=up_max, dn_min=dn_min, delta=delta, lam=lam)


class BrutePLDS:
    def __init__(self, n, delta=Fraction(2, 5), lam=Fraction(3), levels_per_group=0, coeff=None, jump=False):
        self.n = n
        self.jump = jump
        p = exact_params(n, delta, lam, levels_per_group, coeff)
        self.__dict__.update(p)
        self.adj = [set() for _ in range(n)]
        self.level = [0] * n
        self.sweeps_ins = self.sweeps_del = 0

    # degrees as if v sat at level lv
    def cnt_ge(self, v, j):
        return sum(1 for w in self.adj[v] if self.level[w] >= j)

    def inv1_ok(self, v, lv):
        return self.cnt_ge(v, lv) <= self.up_max[lv // self.L]

    def inv2_ok(self, v, lv):
        return lv == 0 or self.cnt_ge(v, lv - 1) >= self.dn_min[(lv - 1) // self.L]

    def desire_level(self, v):
        """Def. desire-level: the level closest to level(v) where both
        invariants hold (all K levels tried)."""
        best = None
        for lp in range(self.K):
            if self.inv1_ok(v, lp) and self.inv2_ok(v, lp):
                dist = abs(lp - self.level[v])
                if best is None or dist < best[0]:
                    best = (dist, lp)
                elif dist == best[0]:
                    raise AssertionError("desire-level not unique")
        return best[1]

    def update(self, ins=(), dele=()):
        for (a, b) in list(ins) + list(dele):
            if not (0 <= a < self.n and 0 <= b < self.n):
                return -2
        self.sweeps_ins = self.sweeps_del = 0
        added = False
        for (a, b) in ins:
            if a != b and b not in self.adj[a]:
                self.adj[a].add(b)
                self.adj[b].add(a)
                added = True
        if added:
            for l in range(self.K):
                S = [v for v in range(self.n) if self.level[v] == l and not self.inv1_ok(v, l)]
                if S:
                    self.sweeps_ins += 1
                    target = {v: (self.desire_level(v) if self.jump else l + 1) for v in S}
                    assert all(t > l for t in target.values())
                    for v in S:
                        self.level[v] = target[v]
        removed = False
        for (a, b) in dele:
            if a != b and b in self.adj[a]:
                self.adj[a].discard(b)
                self.adj[b].discard(a)
                removed = True
        if removed:
            for l in range(self.K):
                viol = [v for v in range(self.n) if not self.inv2_ok(v, self.level[v])]
                dls = {v: self.desire_level(v) for v in viol}
                assert all(d >= l for d in dls.values())
                D = [v for v, d in dls.items() if d == l]
                if D:
                    self.sweeps_del += 1
                    for v in D:
                        self.level[v] = l
        return 0

    def invariants_hold(self):
        return all(self.inv1_ok(v, self.level[v]) and self.inv2_ok(v, self.level[v]) for v in range(self.n))

    def estimate(self, v):
        """Def. coreness estimate, 0 for isolated vertices."""
        if not self.adj[v]:
            return Fraction(0)
        e = max((self.level[v] + 1) // self.L - 1, 0)
        return (1 + self.delta) ** e


def kcore_by_definition(n, edges):
    """Coreness from the definition: the k-core is what remains after
    repeatedly deleting vertices of degree < k; coreness(v) is the largest k
    whose k-core contains v."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    core = [0] * n
    k = 1
    while True:
        alive = set(range(n))
        changed = True
        while changed:
            changed = False
            for v in list(alive):
                if sum(1 for w in adj[v] if w in alive) < k:
                    alive.discard(v)
                    changed = True
        if not alive:
            return core
        for v in alive:
            core[v] = k
        k += 1
