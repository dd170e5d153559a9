"""Serving J/K builds on one GPU: continuous batching of requests.

A request is a new system (basis) with a sequence of density updates.  Its
plan (pair data, Schwarz factors, class lists) is built once at admission
and reused for every update; update k + 1 is sent only when update k has
returned (closed loop).  Requests are admitted first come, first served,
while their plans fit the HBM budget and the number of active requests is
below a cap; a plan is freed when its request finishes.  The updates of
different requests run concurrently on a small set of device streams.

The scheduler (Server) is host logic over an executor interface, so its
rules are testable with a simulated executor; GpuExecutor drives the C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from .counts import unique_eris


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the run
    basis: object                  # workloads.Basis (or anything the executor accepts)
    densities: list                # one N x N array per update
    tau: float = 1e-12
    theta: float = 0.0             # > tau: mixed-precision plan


@dataclasses.dataclass
class UpdateRecord:
    rid: int
    k: int
    submit: float
    done: float

    @property
    def latency(self):
        return self.done - self.submit


@dataclasses.dataclass
class RequestRecord:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    plan_bytes: int = 0
    rejected: str | None = None

    @property
    def latency(self):
        return self.finished - self.arrival


class OverBudget(Exception):
    """The plan does not fit the HBM left right now."""


class TooLarge(Exception):
    """The plan does not fit the whole HBM budget: the request is rejected."""


class Server:
    """Continuous batching: admit, submit, complete, release.

    executor must provide now(), create(request, bytes_left) -> handle
    (raising OverBudget or TooLarge), plan_bytes(handle), submit(handle,
    request, k, slot) -> token, done(token) -> bool, finish(token, request,
    k), release(handle) and idle(until) (wait for progress, at most until
    the given time).  An executor that also has create_async(request,
    bytes_left) -> future (done(), result()) builds plans off the scheduling
    loop, one at a time, so updates keep flowing meanwhile; a plan in the
    making counts against the budget only once it exists."""

    def __init__(self, executor, hbm_budget: int, max_active: int = 8, slots: int = 4):
        if hbm_budget <= 0 or max_active < 1 or slots < 1:
            raise ValueError("need hbm_budget > 0, max_active >= 1, slots >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.slots = slots
        self.peak_bytes = 0
        self.peak_active = 0

    def run(self, requests):
        ex = self.ex
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting = collections.deque()
        active = collections.OrderedDict()        # rid -> [request, handle, k, token, slot, submit time]
        recs = {r.rid: RequestRecord(r.rid, r.arrival) for r in requests}
        updates = []
        used = 0
        blocked_at = None                         # bytes in use when admission last hit the budget
        nslot = 0
        creating = None                           # (future, request) of the plan being built off the loop
        use_async = hasattr(ex, "create_async")
        t0 = ex.now()

        def admitted(r, h):
            nonlocal used, nslot
            b = ex.plan_bytes(h)
            used += b
            self.peak_bytes = max(self.peak_bytes, used)
            recs[r.rid].admitted = ex.now() - t0
            recs[r.rid].plan_bytes = b
            active[r.rid] = [r, h, 0, None, nslot % self.slots, 0.0]
            nslot += 1

        def refused(r, e, fits_later):
            # OverBudget with plans alive: wait at the head for a release; else reject
            nonlocal blocked_at
            if isinstance(e, OverBudget) and fits_later:
                blocked_at = used
                return False
            waiting.popleft()
            recs[r.rid].rejected = (str(e) if isinstance(e, TooLarge) and str(e) else "plan exceeds the HBM budget")
            return True

        while pending or waiting or active or creating:
            t = ex.now() - t0
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            if creating is not None and creating[0].done():
                fut, r = creating
                creating = None
                try:
                    h = fut.result()
                except (OverBudget, TooLarge) as e:
                    refused(r, e, bool(active))
                else:
                    waiting.popleft()
                    admitted(r, h)
            # admission: first come, first served; a request that does not fit now
            # waits at the head until a release frees HBM
            while (creating is None and waiting and len(active) < self.max_active and blocked_at != used):
                r = waiting[0]
                if not r.densities:
                    waiting.popleft()
                    recs[r.rid].admitted = recs[r.rid].finished = ex.now() - t0
                    continue
                if used >= self.budget:
                    if refused(r, OverBudget(), bool(active)):
                        continue
                    break
                if use_async:
                    creating = (ex.create_async(r, self.budget - used), r)
                    break
                try:
                    h = ex.create(r, self.budget - used)
                except (OverBudget, TooLarge) as e:
                    if refused(r, e, bool(active)):
                        continue
                    break
                waiting.popleft()
                admitted(r, h)
            self.peak_active = max(self.peak_active, len(active))
            # closed loop: each active request has at most one update in flight
            for st in active.values():
                if st[3] is None:
                    st[5] = ex.now() - t0
                    st[3] = ex.submit(st[1], st[0], st[2], st[4])
            # completions
            progressed = False
            for rid in list(active):
                st = active[rid]
                if not ex.done(st[3]):
                    continue
                progressed = True
                tdone = ex.now() - t0
                ex.finish(st[3], st[0], st[2])
                updates.append(UpdateRecord(rid, st[2], st[5], tdone))
                st[2] += 1
                st[3] = None
                if st[2] == len(st[0].densities):
                    ex.release(st[1])
                    used -= recs[rid].plan_bytes
                    recs[rid].finished = tdone
                    del active[rid]
            if not progressed:
                nxt = pending[0].arrival + t0 if pending else None
                if active or creating or nxt is not None:
                    ex.idle(nxt)
        return [recs[r.rid] for r in requests], updates


class IterationServer:
    """Iteration-level batching over one multi-system plan.

    Each step runs the next update of every active request together, as one
    J/K build of a plan over all their systems (each class one launch over
    the quartets of every system).  When the active set changes, the plan
    is rebuilt for the new set.  Admission is first come, first served
    under max_active; a plan that exceeds the HBM budget sends the most
    recently admitted requests back to the head of the queue, and a request
    that cannot fit even alone is rejected.

    executor must provide now(), build(requests, budget) -> plan (raising
    OverBudget), submit(plan, requests, ks) -> token, done(token),
    finish(token, requests, ks), release(plan) and idle(until); drop(request),
    if it has one, is called when a request leaves the active set unfinished
    (sent back to the queue or rejected) so that it can free the request's
    device data."""

    def __init__(self, executor, hbm_budget: int, max_active: int = 16):
        if hbm_budget <= 0 or max_active < 1:
            raise ValueError("need hbm_budget > 0, max_active >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.peak_active = 0
        self.rebuilds = 0

    def run(self, requests):
        ex = self.ex
        drop = getattr(ex, "drop", lambda r: None)
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting = collections.deque()
        active = []                               # [request, k]
        recs = {r.rid: RequestRecord(r.rid, r.arrival) for r in requests}
        updates = []
        plan = None
        t0 = ex.now()
        while pending or waiting or active:
            t = ex.now() - t0
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            changed = plan is None
            while waiting and len(active) < self.max_active:
                r = waiting.popleft()
                if not r.densities:
                    recs[r.rid].admitted = recs[r.rid].finished = t
                    continue
                active.append([r, 0])
                recs[r.rid].admitted = t
                changed = True
            if not active:
                if pending:
                    ex.idle(pending[0].arrival + t0)
                continue
            if changed:
                if plan is not None:
                    ex.release(plan)
                    plan = None
                while plan is None:
                    try:
                        plan = ex.build([a[0] for a in active], self.budget)
                    except OverBudget:
                        if len(active) == 1:          # cannot fit even alone
                            r = active.pop()[0]
                            recs[r.rid].rejected = "plan exceeds the HBM budget"
                            recs[r.rid].admitted = float("nan")
                            drop(r)
                            if not active:
                                break
                            continue
                        r = active.pop()[0]           # the latest admitted waits again, at the head
                        recs[r.rid].admitted = float("nan")
                        drop(r)                       # its device data is made again when it is next planned
                        waiting.appendleft(r)
                if plan is None:
                    continue
                self.rebuilds += 1
            self.peak_active = max(self.peak_active, len(active))
            reqs = [a[0] for a in active]
            ks = [a[1] for a in active]
            ts = ex.now() - t0
            tok = ex.submit(plan, reqs, ks)
            while not ex.done(tok):
                ex.idle(None)
            td = ex.now() - t0
            ex.finish(tok, reqs, ks)
            still = []
            for a in active:
                updates.append(UpdateRecord(a[0].rid, a[1], ts, td))
                a[1] += 1
                if a[1] == len(a[0].densities):
                    recs[a[0].rid].finished = td
                else:
                    still.append(a)
            if len(still) != len(active):
                active = still
                if plan is not None and not active:
                    ex.release(plan)
                    plan = None
                elif plan is not None:
                    ex.release(plan)                   # the set changed: rebuild at the next step
                    plan = None
        if plan is not None:
            ex.release(plan)
        return [recs[r.rid] for r in requests], updates


def percentile(x, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    v = np.sort(np.asarray(x, dtype=float))
    if v.size == 0:
        raise ValueError("empty sample")
    k = int(np.ceil(q / 100.0 * v.size)) - 1
    return float(v[min(max(k, 0), v.size - 1)])


def summarize(reqs, updates, elapsed):
    done = [r for r in reqs if r.rejected is None]
    lat_u = [u.latency for u in updates]
    lat_r = [r.latency for r in done]
    span = max(r.arrival for r in reqs) if reqs else 0.0
    return {
        "requests": len(reqs), "rejected": len(reqs) - len(done), "updates": len(updates),
        "elapsed_s": elapsed,
        "offered_req_per_s": (len(reqs) - 1) / span if span > 0 else None,
        "achieved_req_per_s": len(done) / elapsed if elapsed > 0 else None,
        "updates_per_s": len(updates) / elapsed if elapsed > 0 else None,
        "update_p50_ms": 1e3 * percentile(lat_u, 50) if lat_u else None,
        "update_p99_ms": 1e3 * percentile(lat_u, 99) if lat_u else None,
        "request_p50_ms": 1e3 * percentile(lat_r, 50) if lat_r else None,
        "request_p99_ms": 1e3 * percentile(lat_r, 99) if lat_r else None,
    }


def poisson_arrivals(rate: float, n: int, seed: int):
    """n arrival times (s) of a Poisson process of the given rate, the first at 0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


class GpuExecutor:
    """Runs the plans through the C ABI on `slots` device streams.

    Densities are copied to the device at admission (the request's inputs
    then stay resident); each update writes the request's J and K buffers.
    keep(rid, k) -> bool selects updates whose J and K are copied back to
    the host and kept in self.results[(rid, k)] (True: all of them).
    self.eris[rid] is the number of contracted ERIs one update evaluates."""

    def __init__(self, slots: int = 4, keep=False, worker: bool = False):
        import concurrent.futures
        import torch
        from . import lib
        lib()
        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        # worker=True builds and destroys plans on a worker thread, so the
        # loop keeps feeding the streams meanwhile.  Freeing device memory
        # waits for the whole device, though, so a worker's plans arrive
        # slower than the loop's own and fewer requests are active: measured
        # on the serving benchmark, 4.1 against 6.1 updates/s.  Off by default.
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=1) if worker else None
        if worker:
            self.create_async = lambda r, left: self.pool.submit(self.create, r, left)
        self.keep = (lambda rid, k: True) if keep is True else (keep or (lambda rid, k: False))
        self.results = {}
        self.eris = {}

    def now(self):
        return time.perf_counter()

    def create(self, r, bytes_left):
        from . import HGPError, STATUS_OOM, Basis, Plan
        torch = self.torch
        n = int(np.asarray(r.densities[0]).shape[0])
        dev_bytes = 8 * n * n * (len(r.densities) + 2)          # densities, J, K
        if dev_bytes >= bytes_left:
            raise OverBudget()
        b = Basis.from_workload(r.basis)
        try:
            p = Plan(b, tau=r.tau, hbm_budget=int(bytes_left - dev_bytes), theta=r.theta)
        except HGPError as e:
            b.close()
            if e.status == STATUS_OOM:
                raise OverBudget() from e
            raise
        D = [torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda") for x in r.densities]
        J = torch.empty_like(D[0])
        K = torch.empty_like(D[0])
        self.eris[r.rid] = unique_eris(p.schwarz(), np.asarray(r.basis.l), r.tau)[0]
        return {"basis": b, "plan": p, "D": D, "J": J, "K": K, "bytes": p.stats()["device_bytes"] + dev_bytes}

    def plan_bytes(self, h):
        return h["bytes"]

    def submit(self, h, r, k, slot):
        s = self.streams[slot]
        h["plan"].jk(h["D"][k], h["J"], h["K"], stream=s)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return (ev, h)

    def done(self, token):
        return token[0].query()

    def finish(self, token, r, k):
        if self.keep(r.rid, k):
            h = token[1]
            self.results[(r.rid, k)] = (h["J"].cpu().numpy(), h["K"].cpu().numpy())

    def release(self, h):
        # the request's last update has completed, so nothing in flight uses these
        def free():
            h["plan"].close()
            h["basis"].close()
            h["D"] = h["J"] = h["K"] = None
        if self.pool is not None:
            self.pool.submit(free)
        else:
            free()

    def idle(self, until):
        time.sleep(50e-6)

    def close(self):
        if self.pool is not None:
            self.pool.shutdown(wait=True)


class GpuMultiExecutor:
    """IterationServer's executor: one multi-system plan per active set
    (hgp_plan_create_multi / hgp_jk_multi).  A request's densities are put
    on the device when it is first planned and stay there until it
    finishes; keep(rid, k) as for GpuExecutor.  eris_done counts the
    contracted ERIs of all completed steps."""

    def __init__(self, keep=False, stream=None):
        import torch
        from . import lib
        lib()
        self.torch = torch
        self.stream = stream
        self.keep = (lambda rid, k: True) if keep is True else (keep or (lambda rid, k: False))
        self.results = {}
        self.plan_eris = {}
        self.eris_done = 0                 # contracted ERIs of all completed steps
        self.dev = {}                      # rid -> (basis, [D], J, K)

    def now(self):
        return time.perf_counter()

    def _device(self, r):
        from . import Basis
        torch = self.torch
        if r.rid not in self.dev:
            D = [torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda") for x in r.densities]
            self.dev[r.rid] = (Basis.from_workload(r.basis), D, torch.empty_like(D[0]), torch.empty_like(D[0]))
        return self.dev[r.rid]

    @staticmethod
    def _bytes(r):
        """Device bytes of a request's densities and its J, K buffers."""
        n = int(np.asarray(r.densities[0]).shape[0])
        return 8 * n * n * (len(r.densities) + 2)

    def build(self, reqs, budget):
        """One multi-system plan over `reqs` within `budget`, charging the
        densities and J/K buffers of exactly these requests."""
        from . import HGPError, STATUS_OOM, Plan
        held = sum(self._bytes(r) for r in reqs)
        if held >= budget:
            raise OverBudget()
        devs = [self._device(r) for r in reqs]
        try:
            p = Plan.multi([d[0] for d in devs], tau=reqs[0].tau, theta=reqs[0].theta, hbm_budget=budget - held,
                           stream=self.stream)
        except HGPError as e:
            if e.status == STATUS_OOM:
                raise OverBudget() from e
            raise
        # per system: a multi-system plan pairs no shells of different systems
        Q = p.schwarz()
        n0, eris = 0, 0
        for r in reqs:
            n1 = n0 + len(r.basis.l)
            eris += unique_eris(Q[n0:n1, n0:n1], np.asarray(r.basis.l), r.tau)[0]
            n0 = n1
        self.plan_eris[id(p)] = eris
        return p

    def submit(self, p, reqs, ks):
        devs = [self.dev[r.rid] for r in reqs]
        p.jk_multi([d[1][k] for d, k in zip(devs, ks)], [d[2] for d in devs], [d[3] for d in devs],
                   stream=self.stream)
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream() if self.stream is None else self.stream)
        return (ev, self.plan_eris[id(p)])

    def done(self, token):
        return token[0].query()

    def finish(self, token, reqs, ks):
        self.eris_done += token[1]
        for r, k in zip(reqs, ks):
            d = self.dev[r.rid]
            if self.keep(r.rid, k):
                self.results[(r.rid, k)] = (d[2].cpu().numpy(), d[3].cpu().numpy())
            if k == len(r.densities) - 1:
                d[0].close()
                del self.dev[r.rid]

    def release(self, p):
        self.plan_eris.pop(id(p), None)
        p.close()

    def drop(self, r):
        """Free the device data of a request that left the active set unfinished."""
        d = self.dev.pop(r.rid, None)
        if d is not None:
            d[0].close()

    def idle(self, until):
        time.sleep(50e-6)

    def close(self):
        for d in self.dev.values():
            d[0].close()
        self.dev.clear()
