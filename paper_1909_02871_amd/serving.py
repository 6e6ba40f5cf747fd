"""Client side of the serving runtime: replay a request trace in real time.

A trace is a list of requests with arrival times; decode requests carry the
coded packets their sender emits (device pointers) with emission offsets.
The sender is rateless: it emits its packets in order, one per offset, until
the server reports the generation decoded (rank N); packets it would emit
after that are never sent.  Packets lost on the way are simply absent from
the list.  The driver submits each request when its arrival time comes,
pushes each decode's packets as they are emitted, steps the server
continuously and records when each request completes.  A decode whose
sender has run out of packets, and that the server has admitted and given
every packet without reaching rank N, is cancelled after ``starve_s``
seconds.
"""
from __future__ import annotations

import heapq
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
           clock: Callable[[], float] = time.perf_counter, timeout_s: float = 600.0,
           starve_s: float = 1.0) -> List[dict]:
    """Run the trace through `server` in real time; return the completion records.

    `on_done(record)` runs for each completed request before its memory is
    released (e.g. to copy or check the output).  A decode's record also holds
    ``packets_sent``, the packets its sender pushed before completion was
    reported (lost ones not counted)."""
    reqs = sorted(trace, key=lambda r: (r.arrival, r.rid))
    done: List[dict] = []
    t0 = clock()
    i = 0
    outstanding = 0
    sending = []            # heap of (next emission time, rid): decodes still emitting
    cursor = {}             # rid -> index of its next packet
    by_id = {}
    exhausted = {}          # rid -> time its sender ran out of packets
    starved = {}            # rid -> when it was first seen admitted, dry and incomplete
    last_scan = 0.0
    while i < len(reqs) or outstanding:
        now = clock() - t0
        if now > timeout_s:
            raise TimeoutError("serving trace did not finish in %.0f s" % timeout_s)
        while i < len(reqs) and reqs[i].arrival <= now:
            r = reqs[i]
            by_id[r.rid] = r
            if r.kind == "encode":
                server.submit_encode(r.rid, r.C, r.S, r.K, r.N, r.ld_s, r.length, now)
            else:
                server.submit_decode(r.rid, r.N, r.length, now)
                cursor[r.rid] = 0
                if r.packets:
                    heapq.heappush(sending, (r.arrival + r.packets[0][2], r.rid))
                else:
                    exhausted[r.rid] = r.arrival
            outstanding += 1
            i += 1
        # each sender emits the packets whose time has come, while its decode is incomplete
        while sending and sending[0][0] <= now:
            _, rid = heapq.heappop(sending)
            if rid not in cursor:
                continue                      # completed: the sender has stopped
            r, j0 = by_id[rid], cursor[rid]
            j = j0
            while j < len(r.packets) and r.arrival + r.packets[j][2] <= now:
                j += 1
            pk = r.packets[j0:j]
            server.push_packets(rid, [p[0] for p in pk], [p[1] for p in pk], [r.arrival + p[2] for p in pk])
            cursor[rid] = j
            if j < len(r.packets):
                heapq.heappush(sending, (r.arrival + r.packets[j][2], rid))
            else:
                exhausted[rid] = r.arrival + r.packets[-1][2]
        if exhausted and now - last_scan > 0.05:
            # a decode whose sender ran dry is cancelled once it has been admitted, has taken
            # every packet that reached it and still lacks rank N after starve_s
            last_scan = now
            for rid, t_last in list(exhausted.items()):
                if now - t_last <= starve_s:
                    continue
                q = server.query(rid)
                if q["state"] == 1 and q["packets_pending"] == 0:
                    if rid not in starved:
                        starved[rid] = now
                    elif now - starved[rid] > starve_s:
                        server.cancel(rid, now)
                        del exhausted[rid]
                else:
                    starved.pop(rid, None)
        inflight = server.step(now)
        finished = server.poll()
        for d in finished:
            d["latency"] = d["t_done"] - d["t_submit"]
            if d["kind"] == "decode":
                d["packets_sent"] = cursor.pop(d["id"], 0)
                exhausted.pop(d["id"], None)
                starved.pop(d["id"], None)
            if on_done is not None:
                on_done(d)
            server.release(d["id"])
            done.append(d)
        outstanding -= len(finished)
        if not finished and inflight == 0 and outstanding == 0 and i < len(reqs):
            # idle until the next arrival
            wait = reqs[i].arrival - (clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    server.drain(clock() - t0)
    return done
