"""Continuous-batching request loop over a SketchPool.

Requests (insert / delete / query batches of device-resident keys) arrive
from many streams, one SF-sketch per stream.  The loop:

* admits a stream when its first request arrives and the pool's HBM budget
  has a free slot (otherwise the stream waits, first come first served);
* packs the head request of every admitted stream with queued work into the
  next launch -- one request per stream per launch, streams served round
  robin, up to max_launch_keys keys -- while up to max_in_flight earlier
  launches are still on the GPU, so requests that arrive mid-flight join the
  next launch instead of waiting for a queue to drain;
* closes a stream after its last request: its Slim is exported (the transfer
  to the collector) and its slot released for the next stream.

Every request is its own schedule call on its stream's sketch (the pool cuts
it into batches exactly as a lone sketch would), so each stream's result does
not depend on what it was mixed with.  Latency = completion (the launch's
event observed done) - arrival.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

from . import SF_REQ_DELETE, SF_REQ_INSERT, SF_REQ_QUERY, SketchPool


@dataclass
class Served:
    """Per-request outcome."""
    arrival: float
    issued: float = -1.0
    done: float = -1.0
    launch: int = -1


@dataclass
class ServeStats:
    requests: int
    keys: int
    launches: int
    makespan_s: float
    latency_ms: dict
    queue_ms: dict
    keys_per_s: float
    mean_requests_per_launch: float
    peak_resident: int
    latency_by_kind_ms: dict = field(default_factory=dict)
    outcomes: list = field(repr=False, default_factory=list)


def _pct(xs, qs=(50, 99)):
    import numpy as np
    if not len(xs):
        return {f"p{q}": None for q in qs}
    a = np.asarray(xs)
    return {f"p{q}": round(float(np.percentile(a, q)) * 1e3, 3) for q in qs} | {"mean": round(float(a.mean()) * 1e3, 3)}


class Server:
    def __init__(self, pool: SketchPool, max_launch_keys: int = 1 << 24, max_in_flight: int = 2):
        self.pool = pool
        self.max_launch_keys = max_launch_keys
        self.max_in_flight = max_in_flight

    def run(self, requests, key_of, out_of=None, export_to=None, realtime: bool = True,
            clock=time.perf_counter) -> ServeStats:
        """requests: objects with .stream .seq .kind .n .arrival .last, sorted by arrival.
        key_of(r) -> device key tensor of r; out_of(r) -> device answer tensor (queries);
        export_to(stream) -> device uint16 tensor for the closing Slim, or None to skip.
        realtime=False makes every request visible at once (saturation)."""
        pool = self.pool
        N = len(requests)
        outcomes = [Served(r.arrival if realtime else 0.0) for r in requests]
        queues: dict[int, deque] = {}
        slot_of: dict[int, int] = {}
        waiting: deque = deque()       # streams waiting for a slot
        ready: deque = deque()         # admitted streams with queued requests, round robin
        in_ready: set = set()
        in_flight: deque = deque()     # (ticket, [request indices])
        nxt = 0
        completed = 0
        launches = 0
        keys_total = 0
        peak = 0
        t0 = clock()

        def now():
            return clock() - t0

        while completed < N:
            progressed = False
            tn = now()
            # arrivals
            while nxt < N and (not realtime or requests[nxt].arrival <= tn):
                r = requests[nxt]
                q = queues.setdefault(r.stream, deque())
                q.append(nxt)
                if r.stream in slot_of:
                    if r.stream not in in_ready:
                        ready.append(r.stream)
                        in_ready.add(r.stream)
                elif len(q) == 1 and r.stream not in waiting:
                    waiting.append(r.stream)
                nxt += 1
                progressed = True
            # completions, in launch order
            while in_flight and pool.done(in_flight[0][0]):
                _, idxs = in_flight.popleft()
                td = now()
                for i in idxs:
                    outcomes[i].done = td
                completed += len(idxs)
                progressed = True
            # admission under the HBM budget
            while waiting:
                slot = pool.acquire()
                if slot is None:
                    break
                st = waiting.popleft()
                slot_of[st] = slot
                peak = max(peak, len(slot_of))
                ready.append(st)
                in_ready.add(st)
                progressed = True
            # next launch
            if ready and len(in_flight) < self.max_in_flight:
                batch, keys, closing = [], 0, []
                rotate = []
                while ready:
                    st = ready[0]
                    i = queues[st][0]
                    r = requests[i]
                    if batch and keys + r.n > self.max_launch_keys:
                        break
                    ready.popleft()
                    queues[st].popleft()
                    batch.append(i)
                    keys += r.n
                    if r.last:
                        closing.append(st)
                    if queues[st] and not r.last:
                        rotate.append(st)
                    else:
                        in_ready.discard(st)
                for st in rotate:
                    ready.append(st)
                launch_reqs = []
                for i in batch:
                    r = requests[i]
                    launch_reqs.append((slot_of[r.stream], r.kind, key_of(r), None,
                                        out_of(r) if r.kind == SF_REQ_QUERY else None))
                ticket = pool.launch(launch_reqs)
                ti = now()
                for i in batch:
                    outcomes[i].issued = ti
                    outcomes[i].launch = launches
                for st in closing:
                    dst = export_to(st) if export_to else None
                    if dst is not None:
                        pool.export_slim(slot_of[st], dst, asynchronous=True)
                    pool.release(slot_of.pop(st))
                in_flight.append((ticket, batch))
                launches += 1
                keys_total += keys
                continue
            if not progressed:
                if in_flight:
                    time.sleep(20e-6)
                elif nxt < N and realtime:
                    time.sleep(max(0.0, min(1e-3, requests[nxt].arrival - now())))
        makespan = now()
        lat = [o.done - o.arrival for o in outcomes]
        qd = [o.issued - o.arrival for o in outcomes]
        by_kind = {}
        for r, o in zip(requests, outcomes):
            by_kind.setdefault(kinds_name(r.kind), []).append(o.done - o.arrival)
        return ServeStats(N, keys_total, launches, makespan, _pct(lat), _pct(qd),
                          keys_total / makespan if makespan > 0 else 0.0,
                          N / max(1, launches), peak, {k: _pct(v) for k, v in sorted(by_kind.items())},
                          outcomes)


def kinds_name(k: int) -> str:
    return {SF_REQ_INSERT: "insert", SF_REQ_DELETE: "delete", SF_REQ_QUERY: "query"}.get(k, "update")
