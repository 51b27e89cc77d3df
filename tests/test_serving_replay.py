"""Host logic of the request loop (paper_1511_06441_amd/serving.py) against a
stand-in server: arrivals are submitted at their times, every completion is
collected once, latency is finish minus arrival, and a stuck server ends in
a TimeoutError instead of a hang."""
import time
from dataclasses import dataclass

import numpy as np
import pytest

from paper_1511_06441_amd import serving


@dataclass
class _Done:
    tag: int


class _FakeServer:
    """Completes each request `delay` seconds after its submission."""

    def __init__(self, delay=0.01, stuck=False):
        self.delay = delay
        self.stuck = stuck
        self.pending = []
        self.submitted = []

    def submit(self, dev, reconstruct=True, tag=0):
        self.submitted.append((tag, time.perf_counter(), reconstruct))
        self.pending.append((time.perf_counter() + self.delay, tag))

    def poll(self):
        if self.stuck:
            return []
        now = time.perf_counter()
        out = [_Done(t) for due, t in self.pending if due <= now]
        self.pending = [(due, t) for due, t in self.pending if due > now]
        return out


def test_closed_loop_collects_every_request_once():
    srv = _FakeServer(delay=0.005)
    tr = serving.replay(srv, list(range(6)), reconstruct=False)
    assert sorted(tr.completions) == list(range(6))
    assert [t for t, _, _ in srv.submitted] == list(range(6))
    assert all(r is False for _, _, r in srv.submitted)
    assert np.all(tr.latency >= 0.004)
    assert tr.makespan >= 0.004


def test_open_loop_respects_arrival_times():
    arrivals = np.array([0.0, 0.03, 0.06])
    srv = _FakeServer(delay=0.002)
    tr = serving.replay(srv, [None] * 3, arrivals=arrivals)
    assert np.all(tr.submitted >= arrivals - 1e-3)
    assert np.all(tr.finished >= tr.submitted)
    assert tr.percentile(50) < 0.03


def test_stuck_server_times_out():
    srv = _FakeServer(stuck=True)
    with pytest.raises(TimeoutError):
        serving.replay(srv, [None] * 2, timeout_s=0.05)
