"""Client side of libpc2's request server (continuous batching).

Requests (encrypt / aggregate / decrypt vectors of any length) arrive over
time.  The server (pc2_server_*, pc2_serve_*; its admission and launch rules
are csrc/serve_sched.hpp) admits a request when its device memory fits in
the HBM budget, cuts it into element groups (one wavefront's share each) and,
whenever the GPU stream of an operation is idle, launches one persistent
kernel over up to `tick_groups` groups drawn from the admitted requests of
that operation, so requests that arrive while others run join the next
launch and the three operations run concurrently on three streams.  A
request completes when its last group has finished; its latency is
completion time minus arrival time.

`serve_trace` feeds the native server a timed trace of `Request`s;
`percentile` summarises latencies.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, Optional

OPS = ("encrypt", "aggregate", "decrypt")


@dataclass
class Request:
    rid: int
    op: str                 # "encrypt" | "aggregate" | "decrypt"
    length: int             # elements
    arrival: float          # seconds on the client's clock
    K: int = 0              # aggregate: number of ciphertext vectors
    payload: object = None  # the pc2 job dict (op, key, device inputs and output)
    # filled by serve_trace
    admitted: Optional[float] = None    # when it was submitted to the server
    completed: Optional[float] = None   # when the server reported it done
    result: object = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed is None else self.completed - self.arrival


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
