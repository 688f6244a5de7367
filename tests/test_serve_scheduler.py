"""CPU checks of the serving scheduler's policy (no GPU): FIFO order, the
batch-size cap, admission by memory budget, continuous batching across
stream slots, and the request generator's arrival statistics."""
import numpy as np

from paper_2603_27151_amd import serve as SV
from paper_2603_27151_amd import workloads as W


class FakeBackend:
    """Batches finish after `delay` polls; records every launch."""

    def __init__(self, delay=2):
        self.delay = delay
        self.launches = []
        self.t = 0.0

    def launch(self, slot, batch):
        self.launches.append((slot, [t.rid for t in batch]))
        return {"left": self.delay}

    def done(self, h):
        h["left"] -= 1
        return h["left"] < 0

    def finish(self, h, tickets):
        pass

    def clock(self):
        self.t += 1.0
        return self.t


def _tickets(needs):
    return [SV.Ticket(i, 0, None, float(i), n) for i, n in enumerate(needs)]


def _sched(fb, n_slots=2, max_batch=4, budget=100):
    return SV.Scheduler(n_slots, max_batch, budget, fb.launch, fb.done, fb.finish, fb.clock)


def test_fifo_and_batch_cap():
    fb = FakeBackend()
    s = _sched(fb, n_slots=1, max_batch=3, budget=10 ** 9)
    for t in _tickets([1] * 7):
        s.submit(t)
    done = []
    while s.busy:
        done += s.poll()
    assert [r for _, b in fb.launches for r in b] == list(range(7))
    assert [len(b) for _, b in fb.launches] == [3, 3, 1]
    assert [t.rid for t in done] == list(range(7))
    assert all(t.done > 0 for t in done)


def test_memory_budget_limits_batches_and_in_flight_bytes():
    fb = FakeBackend(delay=3)
    s = _sched(fb, n_slots=2, max_batch=8, budget=100)
    for t in _tickets([40, 40, 40, 40, 40]):
        s.submit(t)
    peak = 0
    while s.busy:
        s.poll()
        peak = max(peak, s.in_use)
        assert s.in_use <= 100
    assert peak == 80
    assert all(len(b) <= 2 for _, b in fb.launches)


def test_oversized_request_runs_alone_when_idle():
    fb = FakeBackend()
    s = _sched(fb, n_slots=2, max_batch=4, budget=100)
    for t in _tickets([250, 10, 10]):
        s.submit(t)
    s.poll()
    assert fb.launches[0][1] == [0]
    while s.busy:
        s.poll()
    assert sorted(r for _, b in fb.launches for r in b) == [0, 1, 2]


def test_arrivals_during_a_batch_join_the_next_launch_on_the_other_slot():
    fb = FakeBackend(delay=5)
    s = _sched(fb, n_slots=2, max_batch=8, budget=10 ** 9)
    ts = _tickets([1] * 6)
    s.submit(ts[0])
    s.poll()                       # batch [0] on slot 0
    for t in ts[1:4]:
        s.submit(t)
    s.poll()                       # [1, 2, 3] on slot 1 while slot 0 runs
    assert fb.launches == [(0, [0]), (1, [1, 2, 3])]
    for t in ts[4:]:
        s.submit(t)
    while s.busy:
        s.poll()
    assert fb.launches[2][1] == [4, 5]


def test_request_bytes_counts_outputs_and_setup():
    assert SV.request_bytes(1920, 1080, 100_000) == 1920 * 1080 * 20 + 100_000 * 128


def test_poisson_arrivals_match_the_rate():
    req = W.serving_requests(400.0, 5.0)
    gaps = np.diff([r.arrival_s for r in req])
    assert abs(len(req) / 5.0 - 400.0) < 4 * np.sqrt(400.0 / 5.0)
    assert abs(gaps.mean() - 1 / 400.0) < 0.15 / 400.0
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1       # exponential gaps: CV = 1
    soups = np.bincount([r.soup for r in req], minlength=4)
    assert soups.min() > 0.2 * len(req) / 4 * 3.2 / 4
    res = {(r.view.width, r.view.height) for r in req}
    assert res == set(W.SERVING_RES)
