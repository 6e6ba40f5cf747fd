"""Client side of the serving runtime: replay a request trace in real time.

A trace is a list of requests with arrival times; decode requests carry the
coded packets their sender emits (device pointers) with release offsets.  The
driver submits each request when its arrival time comes, pushes its packets,
steps the server continuously and records when each request completes.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple


@dataclass
class TraceRequest:
    rid: int
    arrival: float                 # seconds from the start of the run
    kind: str                      # "encode" or "decode"
    N: int
    length: int
    # encode: device pointers of C (K x N) and S (N rows, ld_s apart)
    C: int = 0
    S: int = 0
    K: int = 0
    ld_s: int = 0
    # decode: (coefficient pointer, payload pointer, release offset in seconds)
    packets: List[Tuple[int, int, float]] = field(default_factory=list)


def percentile(values: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    v = sorted(values)
    if not v:
        raise ValueError("empty")
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


def replay(server, trace: Sequence[TraceRequest], on_done: Optional[Callable[[dict], None]] = None,
           clock: Callable[[], float] = time.perf_counter, timeout_s: float = 600.0) -> List[dict]:
    """Run the trace through `server` in real time; return the completion records.

    `on_done(record)` runs for each completed request before its memory is
    released (e.g. to copy or check the output)."""
    reqs = sorted(trace, key=lambda r: (r.arrival, r.rid))
    done: List[dict] = []
    t0 = clock()
    i = 0
    outstanding = 0
    while i < len(reqs) or outstanding:
        now = clock() - t0
        if now > timeout_s:
            raise TimeoutError("serving trace did not finish in %.0f s" % timeout_s)
        while i < len(reqs) and reqs[i].arrival <= now:
            r = reqs[i]
            if r.kind == "encode":
                server.submit_encode(r.rid, r.C, r.S, r.K, r.N, r.ld_s, r.length, now)
            else:
                server.submit_decode(r.rid, r.N, r.length, now)
                if r.packets:
                    server.push_packets(r.rid, [p[0] for p in r.packets], [p[1] for p in r.packets],
                                        [r.arrival + p[2] for p in r.packets])
            outstanding += 1
            i += 1
        inflight = server.step(now)
        finished = server.poll()
        now2 = clock() - t0
        for d in finished:
            d["latency"] = d["t_done"] - d["t_submit"]
            if on_done is not None:
                on_done(d)
            server.release(d["id"])
            done.append(d)
        outstanding -= len(finished)
        if not finished and inflight == 0 and i < len(reqs) and outstanding == 0:
            # idle until the next arrival
            wait = reqs[i].arrival - (clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    server.drain(clock() - t0)
    return done
