"""Continuous-batching request loop over a libpilot context.

Frames of several concurrent streams arrive over time.  A stream's frame is
eligible once the stream's previous frame has finished (its result is the
next frame's prior, kept on the device); eligible frames are admitted into
solver slots while slots and the HBM budget allow (pilot_admit returns
EAGAIN otherwise and the frame waits), and every loop turn advances all
admitted frames by one LM pass (pilot_step) and collects finished ones
(pilot_poll).  Frames admitted while others are running join the next pass,
so their work overlaps on the device.

The loop is generic: a request supplies its arrival time and a `prepare`
callback that builds the frame's device inputs given the previous result of
its stream.  It records arrival -> completion latency as observed on the
host.
"""
from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional


@dataclass
class Request:
    stream: int
    t_arrival: float                      # seconds from the start of the run
    prepare: Callable[[Any], tuple]      # prev result (or None) -> (DeviceFrame, DeviceResult, keepalive)
    tag: Any = None


@dataclass
class Completion:
    request: Request
    t_admit: float
    t_done: float
    result: Any
    steps: int

    @property
    def latency(self) -> float:
        return self.t_done - self.request.t_arrival


@dataclass
class RunStats:
    completions: List[Completion] = field(default_factory=list)
    steps: int = 0
    eagain: int = 0
    max_active: int = 0
    max_queue: int = 0
    wall: float = 0.0
    last_arrival: float = 0.0
    # host seconds spent building frames, admitting, enqueueing steps
    # (includes waiting for the step two back) and polling
    host_prepare: float = 0.0
    host_admit: float = 0.0
    host_step: float = 0.0
    host_poll: float = 0.0


class ServingLoop:
    def __init__(self, ctx, clock: Callable[[], float] = time.perf_counter):
        self.ctx = ctx
        self.clock = clock

    def run(self, requests: List[Request], realtime: bool = True,
            on_complete: Optional[Callable[[Completion], None]] = None, pause_gc: bool = True) -> RunStats:
        """Serve `requests` (see the module docstring).  pause_gc: Python's
        cyclic garbage collector is switched off for the run (a full
        collection over the many live request objects stalls the loop for
        tens of milliseconds, every frame in flight then waiting on it) and
        restored afterwards."""
        was_enabled = gc.isenabled()
        if pause_gc:
            gc.collect()
            gc.disable()
        try:
            return self._run(requests, realtime, on_complete)
        finally:
            if pause_gc and was_enabled:
                gc.enable()

    def _run(self, requests, realtime, on_complete) -> RunStats:
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        st = RunStats(last_arrival=reqs[-1].t_arrival if reqs else 0.0)
        queues: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        busy: Dict[int, bool] = collections.defaultdict(bool)
        prev: Dict[int, Any] = {}
        active: Dict[int, tuple] = {}
        t0 = self.clock()
        skipped = [0.0]                                  # idle time jumped over (realtime=False)

        def elapsed():
            return self.clock() - t0 + skipped[0]
        nxt = 0
        while nxt < len(reqs) or any(queues.values()) or active:
            now = elapsed()
            if not realtime and not active and not any(queues.values()) and nxt < len(reqs) \
                    and reqs[nxt].t_arrival > now:
                skipped[0] += reqs[nxt].t_arrival - now  # skip idle time: the clock jumps to the arrival
                now = elapsed()
            while nxt < len(reqs) and reqs[nxt].t_arrival <= now:
                queues[reqs[nxt].stream].append(reqs[nxt])
                nxt += 1
            st.max_queue = max(st.max_queue, sum(len(q) for q in queues.values()))
            # admit the head of every idle stream, oldest arrival first
            heads = sorted((q[0].t_arrival, s) for s, q in queues.items() if q and not busy[s])
            for _, s in heads:
                req = queues[s][0]
                t1 = self.clock()
                df, res, keep = req.prepare(prev.get(s))
                t2 = self.clock()
                slot = self.ctx.admit(df, res)
                st.host_prepare += t2 - t1
                st.host_admit += self.clock() - t2
                if slot is None:
                    st.eagain += 1
                    break                               # no slot or budget: retry after the next pass
                queues[s].popleft()
                busy[s] = True
                active[slot] = (req, df, res, keep, elapsed(), st.steps)
            st.max_active = max(st.max_active, len(active))
            if active:
                t1 = self.clock()
                self.ctx.step()
                st.host_step += self.clock() - t1
                st.steps += 1
            elif nxt < len(reqs) and realtime:
                time.sleep(max(0.0, min(reqs[nxt].t_arrival - elapsed(), 0.002)))
            t1 = self.clock()
            done = [slot for slot in list(active) if self.ctx.poll(slot)]
            st.host_poll += self.clock() - t1
            for slot in done:
                req, df, res, keep, t_adm, s0 = active.pop(slot)
                c = Completion(req, t_adm, elapsed(), res, st.steps - s0)
                st.completions.append(c)
                busy[req.stream] = False
                prev[req.stream] = res
                if on_complete:
                    on_complete(c)
            if not active and not any(queues.values()) and nxt >= len(reqs):
                break
        self.ctx.sync()
        st.wall = elapsed()
        return st
