"""Host-side checks of the continuous-batching scheduler with fake render
workers (no GPU): admission never exceeds the HBM budget, requests that
arrive while a batch runs join a later batch, every request completes, and a
failing backend is reported."""
import math
import threading
import time
import types

import numpy as np
import pytest

serve = pytest.importorskip("paper_2512_20943_amd.serve")


class FakeWorker:
    def __init__(self, delay=0.02, fail_on=None):
        self.delay = delay
        self.instances_per_tile = 100.0
        self.batches = []
        self.fail_on = fail_on
        self.active = 0
        self.threads = []
        self.lock = threading.Lock()
        self.max_active = 0

    def render(self, reqs):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        self.batches.append([r.rid for r in reqs])
        self.threads.append(threading.current_thread())
        time.sleep(self.delay)
        with self.lock:
            self.active -= 1
        if self.fail_on is not None and any(r.rid == self.fail_on for r in reqs):
            raise RuntimeError("injected backend failure")
        return None, [None] * len(reqs)


def fake_seq():
    anchor = types.SimpleNamespace(ld=64 * 100)
    return types.SimpleNamespace(anchor=anchor, n_frames=10)


def trace(n, rate, seed=0):
    return serve.make_trace(n, rate, None, 64, 10, seed, resolutions=((64, 48), (128, 96)))


def test_all_requests_complete_and_batches_form():
    tr = trace(60, 2000.0)
    ws = [FakeWorker(0.01), FakeWorker(0.01)]
    srv = serve.Server(fake_seq(), budget_bytes=1 << 40, max_batch=8, workers=ws)
    srv.run(tr)
    assert all(math.isfinite(r.t_done) and r.t_done >= r.arrival for r in tr)
    ids = sorted(i for w in ws for b in w.batches for i in b)
    assert ids == list(range(60))
    assert max(len(b) for w in ws for b in w.batches) > 1
    assert max(len(b) for w in ws for b in w.batches) <= 8


def test_admission_respects_budget():
    tr = trace(40, 5000.0, 1)
    seq = fake_seq()
    one = max(serve.request_bytes(r, seq.anchor.ld, 100.0) for r in tr)
    budget = int(2.5 * one)
    ws = [FakeWorker(0.005), FakeWorker(0.005)]
    srv = serve.Server(seq, budget_bytes=budget, max_batch=16, workers=ws)
    srv.run(tr)
    assert srv.max_in_flight_bytes <= budget
    assert all(math.isfinite(r.t_done) for r in tr)
    assert max(len(b) for w in ws for b in w.batches) <= 2


def test_requests_arriving_during_a_batch_join_the_next_one():
    tr = serve.make_trace(None, 200.0, 0.3, 64, 10, 2, resolutions=((64, 48),))
    w = FakeWorker(0.05)
    srv = serve.Server(fake_seq(), budget_bytes=1 << 40, max_batch=64, workers=[w])
    srv.run(tr)
    # with one worker busy 50 ms per batch and ~10 arrivals per 50 ms, later
    # batches carry the requests that arrived meanwhile
    sizes = [len(b) for b in w.batches]
    assert sizes[0] >= 1 and max(sizes[1:]) > 1
    order = [i for b in w.batches for i in b]
    assert order == sorted(order), "FIFO order across batches"


def test_injected_backend_failure_is_reported():
    tr = trace(20, 2000.0, 3)
    ws = [FakeWorker(0.005, fail_on=5)]
    srv = serve.Server(fake_seq(), budget_bytes=1 << 40, max_batch=4, workers=ws)
    with pytest.raises(RuntimeError, match="injected"):
        srv.run(tr)
    assert math.isinf(tr[5].t_done)
    assert sum(math.isfinite(r.t_done) for r in tr) >= 16


def test_summary_percentiles():
    tr = trace(10, 100.0)
    for k, r in enumerate(tr):
        r.t_done = r.arrival + 0.001 * (k + 1)
    st = serve.summarize(tr)
    assert st["views"] == 10
    assert abs(st["p50_ms"] - np.percentile(np.arange(1, 11), 50)) < 1e-9


def test_lone_requests_on_an_idle_server_render_on_the_scheduler_thread():
    """Sparse arrivals: every batch holds one request and finds both workers
    idle, so it is rendered on the calling thread; switched off, the worker
    threads render them.  Both ways every request completes in order."""
    tr = serve.make_trace(None, 50.0, 0.3, 64, 10, 4, resolutions=((64, 48),))
    assert len(tr) >= 5
    ws = [FakeWorker(0.001), FakeWorker(0.001)]
    srv = serve.Server(fake_seq(), budget_bytes=1 << 40, max_batch=8, workers=ws)
    srv.run(tr)
    assert all(math.isfinite(r.t_done) and r.t_done >= r.t_start >= r.arrival for r in tr)
    me = threading.current_thread()
    assert all(len(b) == 1 for w in ws for b in w.batches)
    assert all(t is me for w in ws for t in w.threads)

    tr2 = serve.make_trace(None, 50.0, 0.3, 64, 10, 4, resolutions=((64, 48),))
    ws2 = [FakeWorker(0.001), FakeWorker(0.001)]
    srv2 = serve.Server(fake_seq(), budget_bytes=1 << 40, max_batch=8, workers=ws2,
                        inline_singletons=False)
    srv2.run(tr2)
    assert all(math.isfinite(r.t_done) for r in tr2)
    assert all(t is not me for w in ws2 for t in w.threads)
