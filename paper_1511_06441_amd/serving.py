"""Request loop around the libcsp server: replays a stream of arrivals
(open loop) or a backlog (closed loop) and records per-request latency.

Every solve and reconstruction runs in the HIP server; this module only
submits, polls and keeps time.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Trace:
    arrival: np.ndarray            # seconds from the start, per request
    submitted: np.ndarray
    finished: np.ndarray
    completions: dict = field(default_factory=dict)   # tag -> Completion

    @property
    def latency(self) -> np.ndarray:
        return self.finished - self.arrival

    def percentile(self, q: float) -> float:
        return float(np.percentile(self.latency, q))

    @property
    def makespan(self) -> float:
        return float(self.finished.max() - self.arrival.min()) if len(self.finished) else 0.0


def replay(server, devs, arrivals=None, reconstruct=True, timeout_s=600.0, nap_s=0.0002,
           progress=None, progress_every_s=15.0) -> Trace:
    """Submit request k at arrivals[k] seconds after the start (all at once
    when arrivals is None) and poll until every request has completed.
    progress(done, submitted, seconds) is called every progress_every_s."""
    count = len(devs)
    arr = np.zeros(count) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    sub = np.full(count, np.nan)
    fin = np.full(count, np.nan)
    comps = {}
    nxt = 0
    t0 = time.perf_counter()
    t_report = progress_every_s
    while len(comps) < count:
        now = time.perf_counter() - t0
        if progress is not None and now >= t_report:
            progress(len(comps), nxt, now)
            t_report += progress_every_s
        while nxt < count and arr[nxt] <= now:
            server.submit(devs[nxt], reconstruct=reconstruct, tag=nxt)
            sub[nxt] = time.perf_counter() - t0
            nxt += 1
        for c in server.poll():
            fin[c.tag] = time.perf_counter() - t0
            comps[c.tag] = c
        if now > timeout_s:
            raise TimeoutError(f"{count - len(comps)} requests unfinished after {timeout_s} s")
        if nxt < count and len(comps) == nxt:
            # nothing in flight: sleep until the next arrival
            time.sleep(max(0.0, min(arr[nxt] - (time.perf_counter() - t0), 0.002)))
        elif nap_s:
            time.sleep(nap_s)
    return Trace(arr, sub, fin, comps)
