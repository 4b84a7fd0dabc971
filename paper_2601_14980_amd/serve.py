"""Continuous-batching serving loop over libpc2's persistent runners.

Requests (encrypt / aggregate / decrypt vectors of any length) arrive over
time.  A request is admitted when its device memory fits in the HBM budget
(first come, first served); an admitted request is cut into element groups
(one wavefront's share each).  Whenever the GPU stream of an operation is
idle, the scheduler launches ONE persistent kernel over up to `tick_groups`
groups shared among every admitted request of that operation (an equal
slice each, leftovers to the oldest) -- so requests that arrive while others
run join the next launch, long requests do not block short ones, and the
three operations run concurrently on three streams.  A request completes when its last group has finished;
its latency is completion time minus arrival time.

The scheduling logic is independent of the device: `Scheduler` drives an
executor with five methods (`bytes_for`, `admit`, `group_size`, `launch`,
`poll`, `release`), so it is tested on the CPU with a simulated executor and
runs on the GPU with `GpuExecutor`.
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
    def __init__(self, executor, hbm_budget: int, tick_groups: int,
                 clock: Callable[[], float] = time.perf_counter):
        if hbm_budget <= 0 or tick_groups <= 0:
            raise ValueError("budget and tick size must be positive")
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
        while self.waiting and self.used + self.waiting[0].nbytes <= self.budget:
            req = self.waiting.popleft()
            self.ex.admit(req)
            req.admitted = now
            req.groups = -(-req.length // self.ex.group_size(req))
            self.used += req.nbytes
            self.max_used = max(self.max_used, self.used)
            self.active[req.op].append(req)

    # ------------------------------------------------------------- batching
    def _form_tick(self, op: str) -> list:
        """Share the launch among all admitted requests of this op: each gets
        an equal slice first (so a long request cannot starve a short one
        that arrived later), then leftover room goes to the oldest."""
        reqs = [r for r in self.active[op] if r.next_group < r.groups]
        if not reqs:
            return []
        room = self.tick_groups
        take = {r.rid: 0 for r in reqs}
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


# ------------------------------------------------------------ GPU executor
class GpuExecutor:
    """Runs scheduler ticks with pc2_runner_launch on one stream per op.

    Request payloads (device tensors, int32 limb rows):
      encrypt:   {"m": [L, m_limbs], "r": [L, Lk]}        -> result [L, 2Lk]
      aggregate: {"inputs": [K tensors [>= L, 2Lk]]}      -> result [L, 2Lk]
      decrypt:   {"c": [L, 2Lk]}                          -> result [L, Lk]
    """

    def __init__(self, ctx, sk, max_groups: int = 1 << 15, max_jobs: int = 512):
        import torch

        from . import pc2
        self.pc2, self.torch = pc2, torch
        self.ctx, self.sk = ctx, sk
        self.L = sk.L
        self.streams = {op: torch.cuda.Stream() for op in OPS}
        codes = {"encrypt": pc2.PC2_OP_ENCRYPT, "aggregate": pc2.PC2_OP_HOM_SUM,
                 "decrypt": pc2.PC2_OP_DECRYPT}
        self.codes = codes
        self.runners = {op: pc2.Runner(ctx, codes[op], sk.nbits, max_jobs, max_groups)
                        for op in OPS}
        self.gsize = {op: pc2.runner_group_size(sk.public, codes[op]) for op in OPS}

    def group_size(self, req: Request) -> int:
        return self.gsize[req.op]

    def bytes_for(self, req: Request) -> int:
        L, Lk = req.length, self.L
        if req.op == "encrypt":
            return L * (8 + 4 * Lk + 8 * Lk)
        if req.op == "aggregate":
            return L * 8 * Lk * (req.K + 1)
        return L * (8 * Lk + 4 * Lk)

    def admit(self, req: Request) -> None:
        torch = self.torch
        L, Lk = req.length, self.L
        width = Lk if req.op == "decrypt" else 2 * Lk
        req.result = torch.empty((L, width), dtype=torch.int32, device="cuda")

    def _job(self, req: Request):
        pc2 = self.pc2
        p = req.payload
        if req.op == "encrypt":
            return dict(op=pc2.PC2_OP_ENCRYPT, pk=self.sk.public, m=p["m"], r=p["r"],
                        out=req.result)
        if req.op == "aggregate":
            return dict(op=pc2.PC2_OP_HOM_SUM, pk=self.sk.public, inputs=p["inputs"],
                        lengths=None, out=req.result)
        return dict(op=pc2.PC2_OP_DECRYPT, sk=self.sk, c=p["c"], out=req.result)

    def launch(self, op: str, pieces: list):
        torch = self.torch
        st = self.streams[op]
        jobs = [self._job(req) for req, _, _ in pieces]
        first = [f for _, f, _ in pieces]
        ngroups = [n for _, _, n in pieces]
        with torch.cuda.stream(st):
            self.runners[op].launch(jobs, first, ngroups)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def poll(self, handle) -> bool:
        return handle.query()

    def release(self, req: Request) -> None:
        pass  # results stay with the request; inputs belong to the caller

    def close(self) -> None:
        for r in self.runners.values():
            r.close()
