"""The continuous-batching scheduler against a simulated executor on a virtual
clock (CPU): every element group runs exactly once, the HBM budget is never
exceeded, admission is first come first served, late short requests join
running batches, and latency is accounted from arrival."""
from __future__ import annotations

import random

import pytest

from paper_2601_14980_amd.serve import OPS, Request, Scheduler, percentile


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Each op is one in-order stream; a tick of g groups takes g * cost[op]."""

    GROUP = 16
    COST = {"encrypt": 1.0e-3, "aggregate": 0.2e-3, "decrypt": 0.3e-3}

    def __init__(self, clock, budget):
        self.clock = clock
        self.budget = budget
        self.live: dict[int, int] = {}
        self.coverage: dict[int, list[int]] = {}
        self.ticks: list[tuple[str, list]] = []

    def group_size(self, req):
        return self.GROUP

    def bytes_for(self, req):
        return req.length * 100

    def admit(self, req):
        self.live[req.rid] = req.nbytes
        assert sum(self.live.values()) <= self.budget
        self.coverage[req.rid] = []

    def launch(self, op, pieces):
        groups = 0
        for req, first, n in pieces:
            self.coverage[req.rid].extend(range(first, first + n))
            groups += n
        self.ticks.append((op, [(r.rid, f, n) for r, f, n in pieces]))
        return self.clock() + groups * self.COST[op]

    def poll(self, handle):
        return self.clock() >= handle - 1e-12

    def release(self, req):
        del self.live[req.rid]


def run(requests, budget=10**9, tick=64, dt=1e-4, **kw):
    clock = Clock()
    ex = FakeExecutor(clock, budget)
    sch = Scheduler(ex, budget, tick, clock=clock, **kw)

    def idle():
        clock.t += dt

    makespan = sch.run_trace(requests, idle=idle, t0=0.0)
    return sch, ex, makespan


def trace(n, seed=0, rate=2000.0):
    rng = random.Random(seed)
    t, out = 0.0, []
    for i in range(n):
        t += rng.expovariate(rate)
        op = rng.choice(OPS)
        L = int(round(2 ** rng.uniform(8, 14)))
        out.append(Request(rid=i, op=op, length=L, arrival=t,
                           K=rng.randint(2, 8) if op == "aggregate" else 0))
    return out


def test_every_group_exactly_once_and_all_complete():
    reqs = trace(120, seed=1)
    sch, ex, _ = run(reqs)
    assert len(sch.finished) == len(reqs)
    for r in reqs:
        groups = -(-r.length // FakeExecutor.GROUP)
        assert sorted(ex.coverage[r.rid]) == list(range(groups))
        assert r.completed >= r.arrival and r.latency >= 0


def test_budget_and_fifo_admission():
    reqs = trace(80, seed=2)
    budget = 400_000
    big = [r for r in reqs if r.length * 100 > budget]
    sch, ex, _ = run(reqs, budget=budget, policy="fair")
    assert sch.max_used <= budget
    assert {r.rid for r in sch.rejected} == {r.rid for r in big}
    admitted = sorted((r for r in reqs if r.admitted is not None), key=lambda r: r.admitted)
    # first come, first served: admission order follows arrival order
    order = [r.rid for r in sorted(admitted, key=lambda r: (r.admitted, r.arrival))]
    assert order == sorted(order, key=lambda rid: reqs[rid].arrival)


def test_late_short_request_joins_running_batches():
    long = Request(rid=0, op="encrypt", length=16 * 1000, arrival=0.0)
    short = Request(rid=1, op="encrypt", length=16 * 2, arrival=0.005)
    sch, ex, _ = run([long, short], tick=64)
    # the short request completes long before the long one
    assert short.completed < long.completed
    # some launch carries groups of both requests
    assert any(len({rid for rid, _, _ in p}) == 2 for _, p in ex.ticks)


def test_ops_overlap_on_separate_streams():
    reqs = [Request(rid=i, op=op, length=16 * 50, arrival=0.0) for i, op in enumerate(OPS)]
    sch, ex, makespan = run(reqs)
    serial = sum(50 * FakeExecutor.COST[op] for op in OPS)
    assert makespan < serial  # the three operations ran concurrently


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0


def test_bad_arguments():
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(Clock(), 1), 0, 4)
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(Clock(), 1), 10, 4, policy="lifo")
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(Clock(), 1), 10, 4, policy="shortest", max_age=-1.0)


@pytest.mark.parametrize("policy", ["fair", "shortest"])
def test_every_group_once_under_each_policy(policy):
    reqs = trace(120, seed=4)
    sch, ex, _ = run(reqs, policy=policy, max_age=0.05)
    assert len(sch.finished) == len(reqs)
    for r in reqs:
        assert sorted(ex.coverage[r.rid]) == list(range(-(-r.length // FakeExecutor.GROUP)))


def test_shortest_first_orders_by_groups_left():
    """A launch goes to the requests with the fewest groups left, each taking
    all it can; under fair share every request gets a slice."""
    reqs = [Request(rid=0, op="encrypt", length=16 * 100, arrival=0.0),
            Request(rid=1, op="encrypt", length=16 * 6, arrival=0.0),
            Request(rid=2, op="encrypt", length=16 * 2, arrival=0.0)]
    sch, ex, _ = run(reqs, tick=4, policy="shortest", max_age=10.0)
    assert ex.ticks[0] == ("encrypt", [(2, 0, 2), (1, 0, 2)])
    assert ex.ticks[1] == ("encrypt", [(1, 2, 4)])
    assert reqs[2].completed < reqs[1].completed < reqs[0].completed
    reqs = [Request(rid=r.rid, op=r.op, length=r.length, arrival=0.0) for r in reqs]
    sch, ex, _ = run(reqs, tick=4, policy="fair")
    assert {rid for rid, _, _ in ex.ticks[0][1]} == {0, 1, 2}


def test_shortest_first_ages_long_requests():
    """Once past max_age a request goes first, whatever its size."""
    long = Request(rid=0, op="encrypt", length=16 * 40, arrival=0.0)
    shorts = [Request(rid=1 + i, op="encrypt", length=16 * 4, arrival=0.001 * i)
              for i in range(60)]
    sch, ex, _ = run([long] + shorts, tick=4, policy="shortest", max_age=0.02)
    first_long = next(i for i, (_, p) in enumerate(ex.ticks) if any(r == 0 for r, _, _ in p))
    assert ex.ticks[first_long][1][0][0] == 0      # the aged request leads its launch
    assert long.completed < max(r.completed for r in shorts)
    sch, ex, _ = run([Request(rid=r.rid, op=r.op, length=r.length, arrival=r.arrival)
                      for r in [long] + shorts], tick=4, policy="shortest", max_age=100.0)
    assert sch.finished[-1].rid == 0               # never aged: served last


def test_first_fit_admission_with_aging():
    """Shortest first: small requests that fit pass a large one waiting for
    memory, until it has waited max_age; then it holds them back, and the
    budget is never exceeded."""
    budget = 16 * 100 * 100 + 10_000             # one 100-group request and three small
    reqs = [Request(rid=0, op="encrypt", length=16 * 100, arrival=0.0),
            Request(rid=1, op="encrypt", length=16 * 100, arrival=0.0001)]
    reqs += [Request(rid=2 + i, op="encrypt", length=16 * 2, arrival=0.0002 + 0.001 * i)
             for i in range(40)]
    sch, ex, _ = run(reqs, budget=budget, tick=8, policy="shortest", max_age=0.02)
    assert sch.max_used <= budget
    assert len(sch.finished) == len(reqs)
    big2 = reqs[1]
    passed = [r for r in reqs[2:] if r.admitted < big2.admitted]
    late = [r for r in reqs[2:] if r.arrival > big2.arrival + 0.02 + 0.005]
    assert passed                                 # small requests went ahead
    assert all(r.admitted >= big2.admitted for r in late)   # not after it aged
    sch, ex, _ = run([Request(rid=r.rid, op=r.op, length=r.length, arrival=r.arrival)
                      for r in reqs], budget=budget, tick=8, policy="fair")
    order = [r.rid for r in sorted(sch.finished, key=lambda r: (r.admitted, r.rid))]
    assert order == sorted(order)                 # first come, first served
