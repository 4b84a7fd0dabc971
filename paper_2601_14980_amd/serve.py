"""Continuous-batching serving loop over libpc2's persistent runners.

Requests (encrypt / aggregate / decrypt vectors of any length) arrive over
time.  A request is admitted when its device memory fits in the HBM budget
(in arrival order; under the shortest-first policy later requests that fit
may pass one that does not, until it has waited `max_age`); an admitted
request is cut into element groups
(one wavefront's share each).  Whenever the GPU stream of an operation is
idle, the scheduler launches ONE persistent kernel over up to `tick_groups`
groups drawn from the admitted requests of that operation -- shortest
remaining first, except that requests admitted more than `max_age` seconds
ago go first (or, with policy "fair", an equal slice each, leftovers to the
oldest) -- so requests that arrive while others run join the next launch,
long requests do not block short ones, and the three operations run
concurrently on three streams.  A request completes when its last group has
finished; its latency is completion time minus arrival time.

On the device these rules run natively: libpc2's request server
(pc2_server_*, pc2_serve_*) implements the same admission and launch
formation in C++ over its persistent runners, and `serve_trace` feeds it a
timed trace.  `Scheduler` states the same rules over an abstract executor
with six methods (`bytes_for`, `admit`, `group_size`, `launch`, `poll`,
`release`), so that they can be exercised on the CPU with a simulated
executor.
"""
from __future__ import annotations

import heapq
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

OPS = ("encrypt", "aggregate", "decrypt")


@dataclass
class Request:
    rid: int
    op: str                 # "encrypt" | "aggregate" | "decrypt"
    length: int             # elements
    arrival: float          # seconds on the scheduler's clock
    K: int = 0              # aggregate: number of ciphertext vectors
    payload: object = None  # executor-specific inputs
    # filled by the scheduler
    nbytes: int = 0
    groups: int = 0
    next_group: int = 0
    done_groups: int = 0
    admitted: Optional[float] = None
    completed: Optional[float] = None
    result: object = None   # executor-specific outputs

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed is None else self.completed - self.arrival


@dataclass
class Tick:
    op: str
    pieces: list            # [(request, first_group, ngroups)]
    handle: object
    started: float


class Scheduler:
    """policy "shortest" (default): requests take a launch in increasing
    order of the groups they have left, except that those admitted more than
    max_age seconds ago go first, oldest first; "fair": each admitted request
    of an operation gets an equal slice of a launch, leftovers to the oldest."""

    def __init__(self, executor, hbm_budget: int, tick_groups: int,
                 clock: Callable[[], float] = time.perf_counter, policy: str = "shortest",
                 max_age: float = 1.0):
        if hbm_budget <= 0 or tick_groups <= 0:
            raise ValueError("budget and tick size must be positive")
        if policy not in ("fair", "shortest") or not max_age >= 0:
            raise ValueError("policy is 'fair' or 'shortest', max_age >= 0")
        self.policy = policy
        self.max_age = max_age
        self.ex = executor
        self.budget = hbm_budget
        self.tick_groups = tick_groups
        self.clock = clock
        self.used = 0
        self.waiting: deque[Request] = deque()          # arrived, not admitted
        self.active = {op: deque() for op in OPS}        # admitted, groups left
        self.inflight: dict[str, Optional[Tick]] = {op: None for op in OPS}
        self.finished: list[Request] = []
        self.ticks = 0
        self.max_used = 0
        self.rejected: list[Request] = []

    # ------------------------------------------------------------ admission
    def submit(self, req: Request) -> None:
        req.nbytes = self.ex.bytes_for(req)
        if req.nbytes > self.budget:
            self.rejected.append(req)   # could never fit: refused outright
            return
        self.waiting.append(req)

    def _admit(self, now: float) -> None:
        """Fair: first come, first served (a request that does not fit holds
        back those behind it).  Shortest: every waiting request that fits, in
        arrival order, except that one waiting longer than max_age which does
        not fit holds back those behind it."""
        first_fit = self.policy == "shortest"
        keep: deque[Request] = deque()
        while self.waiting:
            req = self.waiting.popleft()
            if self.used + req.nbytes > self.budget:
                if not first_fit or now - req.arrival > self.max_age:
                    keep.append(req)
                    keep.extend(self.waiting)
                    self.waiting.clear()
                    break
                keep.append(req)
                continue
            self.ex.admit(req)
            req.admitted = now
            req.groups = -(-req.length // self.ex.group_size(req))
            self.used += req.nbytes
            self.max_used = max(self.max_used, self.used)
            self.active[req.op].append(req)
        self.waiting = keep

    # ------------------------------------------------------------- batching
    def _form_tick(self, op: str) -> list:
        """Fair: share the launch among all admitted requests of this op, an
        equal slice first (so a long request cannot starve a short one that
        arrived later), then leftover room to the oldest.  Shortest: aged
        requests (oldest first), then the rest by groups left, each taking
        all it can."""
        reqs = [r for r in self.active[op] if r.next_group < r.groups]
        if not reqs:
            return []
        room = self.tick_groups
        take = {r.rid: 0 for r in reqs}
        if self.policy == "shortest":
            now = self.clock()
            aged = lambda r: now - r.admitted > self.max_age
            reqs.sort(key=lambda r: (0, r.admitted) if aged(r) else (1, r.groups - r.next_group))
        else:
            share = max(1, room // len(reqs))
            for r in reqs:
                if room == 0:
                    break
                t = min(share, r.groups - r.next_group, room)
                take[r.rid] = t
                room -= t
        for r in reqs:
            if room == 0:
                break
            t = min(r.groups - r.next_group - take[r.rid], room)
            take[r.rid] += t
            room -= t
        pieces = []
        for r in reqs:
            t = take[r.rid]
            if t:
                pieces.append((r, r.next_group, t))
                r.next_group += t
        return pieces

    def _complete(self, tick: Tick, now: float) -> None:
        for req, _, n in tick.pieces:
            req.done_groups += n
            if req.done_groups == req.groups:
                req.completed = now
                self.active[req.op].remove(req)
                self.ex.release(req)
                self.used -= req.nbytes
                self.finished.append(req)

    def step(self) -> bool:
        """One scheduling pass; returns True while work remains."""
        now = self.clock()
        for op in OPS:
            t = self.inflight[op]
            if t is not None and self.ex.poll(t.handle):
                self._complete(t, now)
                self.inflight[op] = None
        self._admit(now)
        for op in OPS:
            if self.inflight[op] is None:
                pieces = self._form_tick(op)
                if pieces:
                    handle = self.ex.launch(op, pieces)
                    self.inflight[op] = Tick(op, pieces, handle, now)
                    self.ticks += 1
        return bool(self.waiting) or any(self.active[op] for op in OPS)

    def run_trace(self, requests: list[Request], idle: Callable[[], None] = lambda: None,
                  t0: Optional[float] = None) -> float:
        """Feed requests at their arrival times (seconds after t0, default
        now) until all complete; arrival times become absolute.  Returns the
        makespan in clock seconds."""
        start = self.clock() if t0 is None else t0
        for r in requests:
            r.arrival += start
        heap = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(heap)
        while True:
            now = self.clock()
            while heap and heap[0][0] <= now:
                self.submit(heapq.heappop(heap)[2])
            busy = self.step()
            if not heap and not busy:
                break
            idle()
        return self.clock() - start


def percentile(values: list[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not values:
        return float("nan")
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]


# ------------------------------------------------------ native server driver
def serve_trace(server, requests: list[Request], clock: Callable[[], float] = time.perf_counter,
                t0: Optional[float] = None) -> float:
    """Feed requests to a libpc2 request server (pc2.Server) at their arrival
    times (seconds after t0, default now; they become absolute) and record
    when each is seen complete.  Each request's payload is its pc2 job dict
    (op, key, device inputs and output).  Returns the makespan in seconds."""
    start = clock() if t0 is None else t0
    for r in requests:
        r.arrival += start
    order = sorted(requests, key=lambda r: (r.arrival, r.rid))
    live: dict[int, Request] = {}
    i = 0
    while i < len(order) or live:
        now = clock()
        while i < len(order) and order[i].arrival <= now:
            r = order[i]
            live[server.submit(r.payload)] = r
            r.admitted = now
            i += 1
        server.progress()
        ids = server.completed()
        if ids:
            now = clock()
            for rid in ids:
                live.pop(rid).completed = now
    return clock() - start
