"""Phase-1 computation graph: the vertical recurrence (Sec. II-A, Eq. vrr),
its construction under an axis rule (Sec. III-A, Alg. 1) and its ordering
(Sec. III-A, Eq. dsa-score, Eq. peaklive).

A node is (e, f, m): the auxiliary integral [e 0|f 0]^(m).  Base nodes
(0, 0, m) are prefactor * F_m(T).  A bra step along axis i builds (e, f, m)
from e' = e - 1_i:

  PA_i (e',f,m) + WP_i (e',f,m+1)
  + e'_i/(2 zeta) [ (e'-1_i,f,m) - rho/zeta (e'-1_i,f,m+1) ]
  + f_i/(2(zeta+eta)) (e',f-1_i,m+1)

and a ket step is its mirror image with QC, WQ, 1/(2 eta), rho/eta and the
cross term e_i/(2(zeta+eta)) (e-1_i, f', m+1).  The targets are the (e, f, 0)
with la <= |e| <= la+lb and lc <= |f| <= lc+ld, accumulated over primitives
(accumulate-then-transform, Sec. III-C.1, Alg. 2).
"""
from __future__ import annotations

import dataclasses
import heapq

from .cart import add, levels

AXIS_RULES = ("ket_zyx", "bra_xyz", "literal")


@dataclasses.dataclass
class Node:
    key: tuple                 # (e, f, m)
    kind: str                  # 'base' | 'bra' | 'ket'
    axis: int = -1
    parents: tuple = ()        # node ids: (p1, p2, p3|None, p4|None, p5|None)
    k_same: int = 0            # integer factor of the same-side term
    k_cross: int = 0           # integer factor of the cross term


class VRRGraph:
    def __init__(self, la, lb, lc, ld, rule="ket_zyx"):
        assert rule in AXIS_RULES
        self.ls = (la, lb, lc, ld)
        self.L = la + lb + lc + ld
        self.rule = rule
        self.nodes: list[Node] = []
        self.index: dict = {}
        self.targets = [(e, f) for e in levels(la, la + lb) for f in levels(lc, lc + ld)]
        self.target_ids = [self._need((e, f, 0)) for (e, f) in self.targets]
        self.children = [[] for _ in self.nodes]
        for v, nd in enumerate(self.nodes):
            for p in nd.parents:
                if p is not None:
                    self.children[p].append(v)
        self.is_target = [False] * len(self.nodes)
        for t in self.target_ids:
            self.is_target[t] = True

    # -- axis choice -------------------------------------------------------
    def _axis(self, e, f):
        if self.rule == "ket_zyx":
            # consumer-first: reduce the ket index first, z -> y -> x (text reading of Alg. 1)
            for i in (2, 1, 0):
                if f[i] > 0:
                    return "ket", i
            for i in (2, 1, 0):
                if e[i] > 0:
                    return "bra", i
        elif self.rule == "bra_xyz":
            # conventional order: reduce the bra first, x -> y -> z
            for i in (0, 1, 2):
                if e[i] > 0:
                    return "bra", i
            for i in (0, 1, 2):
                if f[i] > 0:
                    return "ket", i
        else:
            # Alg. 1 read literally: the loop keeps overwriting, so the last
            # eligible axis wins (largest i; ket before bra within one axis)
            side = None
            for i in (0, 1, 2):
                if f[i] > 0:
                    side = ("ket", i)
                elif e[i] > 0:
                    side = ("bra", i)
            return side
        raise AssertionError("base node has no axis")

    def _need(self, key):
        if key in self.index:
            return self.index[key]
        e, f, m = key
        if sum(e) == 0 and sum(f) == 0:
            nd = Node(key, "base")
        else:
            side, i = self._axis(e, f)
            if side == "bra":
                e1 = add(e, i, -1)
                p1 = self._need((e1, f, m))
                p2 = self._need((e1, f, m + 1))
                p3 = p4 = p5 = None
                ks = e1[i]
                kc = f[i]
                if ks:
                    e2 = add(e1, i, -1)
                    p3 = self._need((e2, f, m))
                    p4 = self._need((e2, f, m + 1))
                if kc:
                    p5 = self._need((e1, add(f, i, -1), m + 1))
            else:
                f1 = add(f, i, -1)
                p1 = self._need((e, f1, m))
                p2 = self._need((e, f1, m + 1))
                p3 = p4 = p5 = None
                ks = f1[i]
                kc = e[i]
                if ks:
                    f2 = add(f1, i, -1)
                    p3 = self._need((e, f2, m))
                    p4 = self._need((e, f2, m + 1))
                if kc:
                    p5 = self._need((add(e, i, -1), f1, m + 1))
            nd = Node(key, side, i, (p1, p2, p3, p4, p5), ks, kc)
        self.index[key] = len(self.nodes)
        self.nodes.append(nd)
        return self.index[key]

    # -- counts ------------------------------------------------------------
    def flops(self) -> int:
        """FLOPs of the emitted straight-line VRR per primitive quartet: a
        multiply and an FMA for the two leading terms, two FMAs for the
        same-side term, one FMA for the cross term, one multiply per base
        node and one add per accumulated target."""
        n = 0
        for nd in self.nodes:
            if nd.kind == "base":
                n += 1
                continue
            n += 3
            if nd.k_same:
                n += 4
            if nd.k_cross:
                n += 2
        return n + len(self.target_ids)

    def n_hrr(self) -> int:
        return len(self.targets)


# ---------------------------------------------------------------------------
# Orders
# ---------------------------------------------------------------------------

def peak_live(g: VRRGraph, order) -> int:
    """Eq. peaklive: the largest number of computed values that still have an
    unscheduled consumer.  Targets are folded into their accumulators when
    computed, so they stay live only while a consumer remains."""
    pos = {v: t for t, v in enumerate(order)}
    last_use = [-1] * len(g.nodes)
    for v in order:
        for c in g.children[v]:
            last_use[v] = max(last_use[v], pos[c])
    live = 0
    peak = 0
    dies_at = {}
    for t, v in enumerate(order):
        if last_use[v] > t:
            live += 1
            dies_at.setdefault(last_use[v], []).append(v)
        peak = max(peak, live)
        live -= len(dies_at.pop(t, ()))
    return peak


def order_dfs(g: VRRGraph):
    """Post-order depth-first walk from the targets (parents in formula order)."""
    seen = [False] * len(g.nodes)
    out = []
    for t in g.target_ids:
        stack = [(t, 0)]
        while stack:
            v, k = stack.pop()
            if seen[v]:
                continue
            ps = [p for p in g.nodes[v].parents if p is not None]
            if k < len(ps):
                stack.append((v, k + 1))
                if not seen[ps[k]]:
                    stack.append((ps[k], 0))
            else:
                seen[v] = True
                out.append(v)
    return out


def _list_schedule(g: VRRGraph, priority):
    """Generic list scheduler: repeatedly emit the ready node with the
    smallest priority key (priority(v, state) -> tuple)."""
    n = len(g.nodes)
    indeg = [sum(1 for p in set(nd.parents) if p is not None) for nd in g.nodes]
    remaining_uses = [len(set(g.children[v])) for v in range(n)]
    ready = [v for v in range(n) if indeg[v] == 0]
    out = []
    done = [False] * n
    state = {"remaining_uses": remaining_uses}
    while ready:
        best = min(ready, key=lambda v: priority(v, state))
        ready.remove(best)
        out.append(best)
        done[best] = True
        for p in set(g.nodes[best].parents):
            if p is not None:
                remaining_uses[p] -= 1
        for c in set(g.children[best]):
            indeg[c] -= 1
            if indeg[c] == 0:
                ready.append(c)
    assert len(out) == n
    return out


def order_greedy(g: VRRGraph):
    """Free-most greedy: prefer the ready node that retires the most live
    parents (their last use), then the one that adds no long-lived value,
    then the deepest (largest m first), then the lowest id."""
    def prio(v, st):
        ru = st["remaining_uses"]
        frees = sum(1 for p in set(g.nodes[v].parents) if p is not None and ru[p] == 1)
        grows = 1 if g.children[v] else 0
        return (-(frees - grows), -g.nodes[v].key[2], v)
    return _list_schedule(g, prio)


def order_dsa(g: VRRGraph):
    """Eq. dsa-score read statically: score(v) = sum over w in Reach(v) of
    (out(w) - in(w)), with Reach(v) = v and every node reachable from it along
    data-flow edges, out/in the static fan-out/fan-in; ties to the lowest id.
    The ready node with the largest score is emitted next."""
    n = len(g.nodes)
    d = [len(set(g.children[v])) - sum(1 for p in set(g.nodes[v].parents) if p is not None) for v in range(n)]
    topo = order_dfs(g)
    reach = [0] * n
    for v in reversed(topo):
        r = 1 << v
        for c in set(g.children[v]):
            r |= reach[c]
        reach[v] = r
    score = []
    for v in range(n):
        r = reach[v]
        s = 0
        while r:
            low = r & -r
            s += d[low.bit_length() - 1]
            r ^= low
        score.append(s)
    return _list_schedule(g, lambda v, st: (-score[v], v))


def _ancestor_counts(g: VRRGraph):
    anc = [0] * len(g.nodes)
    for v in order_dfs(g):
        r = 1 << v
        for p in g.nodes[v].parents:
            if p is not None:
                r |= anc[p]
        anc[v] = r
    return [bin(a).count("1") for a in anc]


def order_dfs_su(g: VRRGraph, target_key=None):
    """Depth-first post-order that visits the parent with the larger ancestor
    cone first (Sethi-Ullman style), over the targets sorted by target_key
    (default: by the bra component e, then the ket component f)."""
    ac = _ancestor_counts(g)
    key = target_key or (lambda t: (g.nodes[t].key[0], g.nodes[t].key[1]))
    seen = [False] * len(g.nodes)
    out = []
    for t in sorted(g.target_ids, key=key):
        stack = [(t, None)]
        while stack:
            v, ps = stack.pop()
            if seen[v]:
                continue
            if ps is None:
                ps = sorted({p for p in g.nodes[v].parents if p is not None}, key=lambda p: (-ac[p], p))
            ps = [p for p in ps if not seen[p]]
            if ps:
                stack.append((v, ps[1:]))
                stack.append((ps[0], None))
            else:
                seen[v] = True
                out.append(v)
    return out


def order_dfs_su_f(g: VRRGraph):
    return order_dfs_su(g, lambda t: (g.nodes[t].key[1], g.nodes[t].key[0]))


SCHEDULERS = {"dfs": order_dfs, "greedy": order_greedy, "dsa": order_dsa,
              "dfs_su_e": order_dfs_su, "dfs_su_f": order_dfs_su_f}


def best_order(g: VRRGraph, schedulers=("dfs_su_e", "dfs_su_f", "dfs", "greedy", "dsa")):
    """Run each scheduler and keep the order with the smallest PeakLive."""
    best = None
    for name in schedulers:
        if name in ("dsa", "greedy") and len(g.nodes) > 6000:
            continue
        o = SCHEDULERS[name](g)
        pl = peak_live(g, o)
        if best is None or pl < best[1]:
            best = (name, pl, o)
    return best
