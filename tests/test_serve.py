"""The serving scheduler's rules, with a simulated executor (no GPU):
closed-loop updates, first-come-first-served admission under the HBM
budget and the active cap, rejection of plans that cannot fit, and the
latency statistics."""
import numpy as np
import pytest

from paper_2605_10312_amd import serve


class SimExecutor:
    """Simulated clock; each slot runs its updates one at a time in order;
    request r's plan takes bytes[r] and each of its updates cost[r] seconds."""

    def __init__(self, bytes_, cost, create_cost=0.0):
        self.t = 0.0
        self.bytes = bytes_
        self.cost = cost
        self.create_cost = create_cost
        self.slot_free = {}
        self.log = []

    def now(self):
        return self.t

    def create(self, r, left):
        if self.bytes[r.rid] > left:
            raise serve.OverBudget()
        self.t += self.create_cost
        self.log.append(("create", r.rid, self.t, left))
        return r.rid

    def plan_bytes(self, h):
        return self.bytes[h]

    def submit(self, h, r, k, slot):
        start = max(self.t, self.slot_free.get(slot, 0.0))
        end = start + self.cost[h]
        self.slot_free[slot] = end
        self.log.append(("submit", h, k, self.t))
        return end

    def done(self, token):
        return token <= self.t + 1e-12

    def finish(self, token, r, k):
        self.log.append(("finish", r.rid, k, self.t))

    def release(self, h):
        self.log.append(("release", h, self.t))

    def idle(self, until):
        ends = [e for e in self.slot_free.values() if e > self.t + 1e-12]
        cand = ends + ([until] if until is not None and until > self.t else [])
        self.t = min(cand) if cand else self.t + 1e-3


def _reqs(n, nupd, gap=0.01):
    return [serve.Request(i, i * gap, None, [None] * nupd) for i in range(n)]


def test_closed_loop_every_update_in_order():
    reqs = _reqs(6, 4)
    ex = SimExecutor({i: 10 for i in range(6)}, {i: 0.005 * (1 + i % 3) for i in range(6)})
    recs, ups = serve.Server(ex, hbm_budget=1000, max_active=4, slots=2).run(reqs)
    assert all(r.rejected is None for r in recs)
    for i in range(6):
        mine = sorted((u for u in ups if u.rid == i), key=lambda u: u.k)
        assert [u.k for u in mine] == [0, 1, 2, 3]
        for a, b in zip(mine, mine[1:]):
            assert b.submit >= a.done - 1e-12            # update k+1 only after k returned
        assert recs[i].finished == pytest.approx(mine[-1].done)
        assert recs[i].admitted >= recs[i].arrival - 1e-12


def test_budget_and_fcfs_admission():
    reqs = _reqs(8, 3, gap=0.0)
    bytes_ = {i: 40 + 10 * (i % 2) for i in range(8)}
    ex = SimExecutor(bytes_, {i: 0.01 for i in range(8)})
    srv = serve.Server(ex, hbm_budget=100, max_active=8, slots=4)
    recs, ups = srv.run(reqs)
    assert srv.peak_bytes <= 100
    assert srv.peak_active == 2                          # 40 + 50 fits, a third never does
    adm = [r.admitted for r in recs]
    assert adm == sorted(adm)                            # first come, first served
    # at every moment the plans alive fit the budget
    alive = {}
    for ev in ex.log:
        if ev[0] == "create":
            alive[ev[1]] = bytes_[ev[1]]
            assert sum(alive.values()) <= 100
        elif ev[0] == "release":
            del alive[ev[1]]


def test_active_cap_and_rejection():
    reqs = _reqs(5, 2, gap=0.0)
    bytes_ = {0: 10, 1: 500, 2: 10, 3: 10, 4: 10}
    ex = SimExecutor(bytes_, {i: 0.01 for i in range(5)})
    srv = serve.Server(ex, hbm_budget=100, max_active=2, slots=2)
    recs, ups = srv.run(reqs)
    assert recs[1].rejected is not None                  # larger than the whole budget
    assert all(recs[i].rejected is None for i in (0, 2, 3, 4))
    assert srv.peak_active <= 2
    assert len(ups) == 8
    s = serve.summarize(recs, ups, max(u.done for u in ups))
    assert s["rejected"] == 1 and s["updates"] == 8


def test_later_arrivals_wait_for_the_clock():
    reqs = [serve.Request(0, 0.0, None, [None]), serve.Request(1, 5.0, None, [None])]
    ex = SimExecutor({0: 1, 1: 1}, {0: 0.1, 1: 0.1})
    recs, ups = serve.Server(ex, hbm_budget=10).run(reqs)
    assert recs[1].admitted >= 5.0
    assert recs[0].finished == pytest.approx(0.1)
    assert recs[1].latency == pytest.approx(0.1)


def test_percentile_is_nearest_rank():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 100, 1001):
        x = rng.normal(size=n)
        for q in (50, 90, 99, 100):
            assert serve.percentile(x, q) == np.percentile(x, q, method="inverted_cdf")
    with pytest.raises(ValueError):
        serve.percentile([], 50)


def test_poisson_arrivals():
    t = serve.poisson_arrivals(200.0, 20000, seed=1005)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200.0) < 3 * gaps.std() / np.sqrt(gaps.size)
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05    # exponential gaps: CV = 1


class _Future:
    def __init__(self, ex, t_done, fn):
        self.ex, self.t_done, self.fn = ex, t_done, fn

    def done(self):
        return self.ex.t >= self.t_done - 1e-12

    def result(self):
        return self.fn()


class AsyncSimExecutor(SimExecutor):
    """Plans take create_cost seconds to build, off the scheduling loop."""

    def create_async(self, r, left):
        self.log.append(("start", r.rid, self.t, left))

        def fn():
            return self.create(r, left)
        fut = _Future(self, self.t + self.create_cost, fn)
        self.pending_create = fut.t_done
        return fut

    def create(self, r, left):
        if self.bytes[r.rid] > left:
            raise serve.OverBudget()
        self.log.append(("create", r.rid, self.t, left))
        return r.rid

    def idle(self, until):
        c = getattr(self, "pending_create", None)
        if c is not None and c > self.t:
            until = c if until is None else min(until, c)
        super().idle(until)


def test_async_plan_building_overlaps_updates():
    """While a plan is built, the updates of admitted requests keep running;
    the budget and the order of admission still hold."""
    reqs = _reqs(6, 3, gap=0.0)
    bytes_ = {i: 30 for i in range(6)}
    ex = AsyncSimExecutor(bytes_, {i: 0.01 for i in range(6)}, create_cost=0.02)
    srv = serve.Server(ex, hbm_budget=100, max_active=6, slots=3)
    recs, ups = srv.run(reqs)
    assert all(r.rejected is None for r in recs) and len(ups) == 18
    assert srv.peak_bytes <= 100 and 2 <= srv.peak_active <= 3
    adm = [r.admitted for r in recs]
    assert adm == sorted(adm)
    # request 0's updates ran while request 1's plan was being built
    first1 = recs[1].admitted
    assert any(u.rid == 0 and u.done <= first1 + 1e-12 for u in ups)


class IterSimExecutor:
    """Simulated multi-system executor: a step costs the sum of its members'
    costs times `merge` (merged launches are cheaper than separate ones);
    a plan over a set takes the sum of the members' bytes."""

    def __init__(self, bytes_, cost, merge=0.5):
        self.t = 0.0
        self.bytes, self.cost, self.merge = bytes_, cost, merge
        self.end = None
        self.log = []

    def now(self):
        return self.t

    def build(self, reqs, budget):
        if sum(self.bytes[r.rid] for r in reqs) > budget:
            raise serve.OverBudget()
        self.log.append(("build", tuple(r.rid for r in reqs), self.t))
        return tuple(r.rid for r in reqs)

    def submit(self, plan, reqs, ks):
        assert tuple(r.rid for r in reqs) == plan
        self.end = self.t + self.merge * sum(self.cost[r.rid] for r in reqs)
        self.log.append(("step", plan, tuple(ks), self.t))
        return self.end

    def done(self, tok):
        return self.t >= tok - 1e-12

    def finish(self, tok, reqs, ks):
        pass

    def release(self, plan):
        self.log.append(("release", plan, self.t))

    def drop(self, r):
        self.log.append(("drop", r.rid, self.t))

    def idle(self, until):
        if self.end is not None and self.end > self.t:
            self.t = self.end if until is None else min(self.end, until)
        elif until is not None:
            self.t = max(self.t, until)
        else:
            self.t += 1e-3


def test_iteration_server_runs_every_update_once_in_order():
    reqs = [serve.Request(i, 0.01 * i, None, [None] * (2 + i % 3)) for i in range(7)]
    ex = IterSimExecutor({i: 10 for i in range(7)}, {i: 0.004 for i in range(7)})
    srv = serve.IterationServer(ex, hbm_budget=1000, max_active=3)
    recs, ups = srv.run(reqs)
    assert all(r.rejected is None for r in recs)
    assert len(ups) == sum(len(r.densities) for r in reqs)
    for r in reqs:
        mine = sorted((u for u in ups if u.rid == r.rid), key=lambda u: u.submit)
        assert [u.k for u in mine] == list(range(len(r.densities)))     # closed loop, in order
        assert recs[r.rid].finished == pytest.approx(mine[-1].done)
    assert srv.peak_active <= 3
    # every step ran exactly the active set its plan was built for, and plans were rebuilt on change
    steps = [e for e in ex.log if e[0] == "step"]
    assert all(len(e[1]) <= 3 for e in steps) and srv.rebuilds >= 3


def test_iteration_server_budget_pushes_back_and_rejects():
    reqs = [serve.Request(i, 0.0, None, [None] * 2) for i in range(5)]
    bytes_ = {0: 40, 1: 40, 2: 40, 3: 500, 4: 30}
    ex = IterSimExecutor(bytes_, {i: 0.01 for i in range(5)})
    srv = serve.IterationServer(ex, hbm_budget=100, max_active=4)
    recs, ups = srv.run(reqs)
    assert recs[3].rejected is not None
    assert all(recs[i].rejected is None for i in (0, 1, 2, 4))
    for e in ex.log:
        if e[0] == "build":
            assert sum(bytes_[i] for i in e[1]) <= 100
    assert len(ups) == 8
    # the executor is told about every request that leaves the active set unfinished:
    # the rejected one, and each one pushed back to the queue
    drops = [e[1] for e in ex.log if e[0] == "drop"]
    assert 3 in drops
    assert len(drops) >= 2
