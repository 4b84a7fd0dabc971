"""The request server's scheduling rules (csrc/serve_sched.hpp, the code
pc2_server runs) on the CPU: tests/serve_sim.cpp drives them over a virtual
clock and a simulated device (each operation one in-order stream, a launch of
g groups taking g * cost seconds), built here with the host compiler.
Checked: every element group runs exactly once, the HBM budget is never
exceeded, fair-share admission is first come first served, late short
requests join running launches, the three operations overlap, shortest
remaining first orders a launch by groups left, aged requests go first, and
first-fit admission stops passing a request once it has waited the age
limit."""
from __future__ import annotations

import ctypes
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

from paper_2601_14980_amd.serve import percentile

HERE = os.path.dirname(os.path.abspath(__file__))
ENC, AGG, DEC = 0, 1, 2
FAIR, SHORTEST = 0, 1          # PC2_SERVE_FAIR, PC2_SERVE_SHORTEST
GROUP = 16
COST = (1.0e-3, 0.2e-3, 0.3e-3)  # seconds per group: encrypt, aggregate, decrypt


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    out = tmp_path_factory.mktemp("servesim") / "libservesim.so"
    subprocess.run([cxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Werror",
                    "-o", str(out), os.path.join(HERE, "serve_sim.cpp")], check=True)
    so = ctypes.CDLL(str(out))
    d, i64, u64 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), \
        ctypes.POINTER(ctypes.c_uint64)
    so.serve_sim.restype = ctypes.c_long
    so.serve_sim.argtypes = [ctypes.c_int, d, ctypes.POINTER(ctypes.c_int), u64, u64,
                             ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_uint32), d, ctypes.c_double, d, d, i64,
                             ctypes.c_long, u64, d]
    return so


class Run:
    """One simulated trace: per-request admitted / completed times, the
    launches (op, [(request, first group, groups)]), peak admitted bytes."""

    def __init__(self, lib, reqs, budget=10**9, tick=64, policy=SHORTEST, max_age=1.0,
                 dt=1e-4):
        reqs = sorted(reqs, key=lambda r: r["arrival"])
        self.reqs = reqs
        n = len(reqs)
        arr = np.array([r["arrival"] for r in reqs], dtype=np.float64)
        op = np.array([r["op"] for r in reqs], dtype=np.int32)
        cnt = np.array([r["length"] for r in reqs], dtype=np.uint64)
        byt = np.array([r.get("bytes", r["length"] * 100) for r in reqs], dtype=np.uint64)
        ge = np.array([GROUP] * 3, dtype=np.uint32)
        cost = np.array(COST, dtype=np.float64)
        self.admitted = np.zeros(n)
        self.completed = np.zeros(n)
        cap = 1 << 20
        log = np.zeros((cap, 5), dtype=np.int64)
        mu = ctypes.c_uint64()
        ms = ctypes.c_double()
        P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
        rows = lib.serve_sim(n, P(arr, ctypes.c_double), P(op, ctypes.c_int),
                             P(cnt, ctypes.c_uint64), P(byt, ctypes.c_uint64), budget, tick,
                             policy, max_age, P(ge, ctypes.c_uint32),
                             P(cost, ctypes.c_double), dt,
                             P(self.admitted, ctypes.c_double),
                             P(self.completed, ctypes.c_double),
                             P(log, ctypes.c_int64), cap, ctypes.byref(mu), ctypes.byref(ms))
        assert rows != -1, "launch log overflow"
        assert rows != -2, "the trace never finished"
        self.max_used = mu.value
        self.makespan = ms.value
        self.launches: list[tuple[int, list]] = []
        for idx, o, rid, first, g in log[:rows]:
            if idx == len(self.launches):
                self.launches.append((int(o), []))
            self.launches[idx][1].append((int(rid), int(first), int(g)))

    def rid(self, i):
        return self.reqs[i]["rid"]

    def by_rid(self, rid):
        return next(i for i, r in enumerate(self.reqs) if r["rid"] == rid)


def req(rid, op, length, arrival, nbytes=None):
    r = {"rid": rid, "op": op, "length": length, "arrival": arrival}
    if nbytes is not None:
        r["bytes"] = nbytes
    return r


def trace(n, seed=0, rate=2000.0):
    rng = random.Random(seed)
    t, out = 0.0, []
    for i in range(n):
        t += rng.expovariate(rate)
        out.append(req(i, rng.choice((ENC, AGG, DEC)), int(round(2 ** rng.uniform(8, 14))), t))
    return out


def groups_of(r):
    return -(-r["length"] // GROUP)


def coverage(run):
    cov = {i: [] for i in range(len(run.reqs))}
    for _, pieces in run.launches:
        for i, first, g in pieces:
            cov[i].extend(range(first, first + g))
    return cov


@pytest.mark.parametrize("policy", [FAIR, SHORTEST])
def test_every_group_exactly_once_and_all_complete(lib, policy):
    run = Run(lib, trace(120, seed=1), policy=policy, max_age=0.05)
    cov = coverage(run)
    for i, r in enumerate(run.reqs):
        assert sorted(cov[i]) == list(range(groups_of(r)))
        assert run.completed[i] >= run.admitted[i] >= r["arrival"]
    for o, pieces in run.launches:   # a launch holds one op's groups, at most a tick of them
        assert sum(g for _, _, g in pieces) <= 64
        assert {run.reqs[i]["op"] for i, _, _ in pieces} == {o}


def test_budget_and_fifo_admission(lib):
    reqs = trace(80, seed=2)
    budget = 400_000
    run = Run(lib, reqs, budget=budget, policy=FAIR)
    assert run.max_used <= budget
    big = {i for i, r in enumerate(run.reqs) if r["length"] * 100 > budget}
    assert big and all(run.admitted[i] < 0 and run.completed[i] < 0 for i in big)
    ok = [i for i in range(len(run.reqs)) if i not in big]
    # first come, first served: admission times never decrease in arrival order
    times = [run.admitted[i] for i in ok]
    assert times == sorted(times)


def test_late_short_request_joins_running_launches(lib):
    run = Run(lib, [req(0, ENC, 16 * 1000, 0.0), req(1, ENC, 16 * 2, 0.005)], tick=64)
    assert run.completed[1] < run.completed[0]
    assert any(len({i for i, _, _ in p}) == 2 for _, p in run.launches)


def test_ops_overlap_on_separate_streams(lib):
    run = Run(lib, [req(i, op, 16 * 50, 0.0) for i, op in enumerate((ENC, AGG, DEC))])
    serial = sum(50 * c for c in COST)
    assert run.makespan < serial        # the three operations ran concurrently


def test_shortest_first_orders_by_groups_left(lib):
    """A launch goes to the requests with the fewest groups left, each taking
    all it can; under fair share every request gets a slice."""
    reqs = [req(0, ENC, 16 * 100, 0.0), req(1, ENC, 16 * 6, 0.0), req(2, ENC, 16 * 2, 0.0)]
    run = Run(lib, reqs, tick=4, policy=SHORTEST, max_age=10.0)
    assert run.launches[0] == (ENC, [(2, 0, 2), (1, 0, 2)])
    assert run.launches[1] == (ENC, [(1, 2, 4)])
    assert run.completed[2] < run.completed[1] < run.completed[0]
    run = Run(lib, reqs, tick=4, policy=FAIR)
    assert {i for i, _, _ in run.launches[0][1]} == {0, 1, 2}
    assert run.launches[0][1] == [(0, 0, 2), (1, 0, 1), (2, 0, 1)]  # slices, rest to the oldest


def test_shortest_first_ages_long_requests(lib):
    """Once past max_age a request goes first, whatever its size."""
    reqs = [req(0, ENC, 16 * 40, 0.0)] + [req(1 + i, ENC, 16 * 4, 0.001 * i) for i in range(60)]
    run = Run(lib, reqs, tick=4, policy=SHORTEST, max_age=0.02)
    first_long = next(k for k, (_, p) in enumerate(run.launches) if any(i == 0 for i, _, _ in p))
    assert run.launches[first_long][1][0][0] == 0    # the aged request leads its launch
    assert run.completed[0] < run.completed[1:].max()
    run = Run(lib, reqs, tick=4, policy=SHORTEST, max_age=100.0)
    assert run.completed[0] == run.completed.max()   # never aged: served last
    assert run.completed[0] > run.completed[1:].max()


def test_first_fit_admission_with_aging(lib):
    """Shortest first: small requests that fit pass a large one waiting for
    memory, until it has waited max_age; then it holds them back (else the
    stream of small requests would keep it out), and the budget is never
    exceeded.  Fair share admits in arrival order."""
    budget = 170_000                           # the first large request + 3 small, or
    reqs = [req(0, ENC, 16 * 100, 0.0, 160_000),   # the second large one + 1 small
            req(1, ENC, 16 * 100, 0.0001, 166_000)]
    reqs += [req(2 + i, ENC, 16 * 2, 0.0002 + 0.001 * i, 3_200) for i in range(200)]
    run = Run(lib, reqs, budget=budget, tick=8, policy=SHORTEST, max_age=0.02)
    assert run.max_used <= budget
    assert (run.completed > 0).all()
    big2 = 1
    passed = [i for i in range(2, len(reqs)) if run.admitted[i] < run.admitted[big2]]
    late = [i for i in range(2, len(reqs)) if reqs[i]["arrival"] > reqs[big2]["arrival"] + 0.025]
    assert passed                                  # small requests went ahead
    assert all(run.admitted[i] >= run.admitted[big2] for i in late)  # not after it aged
    assert run.admitted[big2] < 0.15               # admitted once the first one finished
    run = Run(lib, reqs, budget=budget, tick=8, policy=FAIR)
    times = list(run.admitted)
    assert times == sorted(times)                  # first come, first served


def test_mixed_trace_accounting(lib):
    """A 2000-request mixed trace under a tight budget: every group once,
    bytes never above the budget, every admitted request completes."""
    reqs = trace(2000, seed=7)
    for r in reqs:
        r["bytes"] = r["length"] * 100
    run = Run(lib, reqs, budget=2_000_000, tick=128, policy=SHORTEST, max_age=0.05, dt=5e-4)
    assert run.max_used <= 2_000_000
    cov = coverage(run)
    for i, r in enumerate(run.reqs):
        assert sorted(cov[i]) == list(range(groups_of(r)))
        assert run.completed[i] > 0


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0
