"""Scheduler of the serving loop on the host: admission by memory, batches
of one eps class in FIFO order, overlap of slots, every request finished.
The device work is replaced by a timed stand-in (no GPU)."""
import threading
import time

import numpy as np
import pytest

pytest.importorskip("torch")
serve = pytest.importorskip("paper_1908_10583_amd.serve")

import synth  # noqa: E402


class FakeRunner:
    def __init__(self, dur=0.02):
        self.dur = dur
        self.lock = threading.Lock()
        self.batches = []
        self.live = 0
        self.max_live = 0

    def __call__(self, batch, stream, nbytes):
        with self.lock:
            self.live += 1
            self.max_live = max(self.max_live, self.live)
            self.batches.append(([r.id for r in batch], {r.eps for r in batch}, nbytes))
        time.sleep(self.dur * (5 if batch[0].eps < 0.3 else 1))
        for r in batch:
            r.ids = np.arange(r.k)
        with self.lock:
            self.live -= 1


def _server(runner, budget, slots=4, max_batch=4):
    return serve.Server(None, slots=slots, max_batch=max_batch, mem_budget=budget,
                        ws_size=lambda b: 100 + 50 * b, runner=runner)


def test_admission_batching_and_overlap():
    trace = synth.poisson_requests(60, 400.0, np.arange(50), seed=3)
    fr = FakeRunner()
    srv = _server(fr, budget=100 + 50 * 4 + 100 + 50 * 2)   # one batch of 4 and one of 2
    reqs = serve.run_trace(srv, trace)
    assert all(r.error is None and r.t_done >= r.t_admit >= r.t_arrival for r in reqs)
    assert sorted(r.id for r in srv.done) == list(range(60))
    assert srv.peak <= srv.budget
    assert fr.max_live >= 2                        # batches overlapped
    for ids, eps, nbytes in fr.batches:
        assert len(eps) == 1                       # one eps class per batch
        assert nbytes == 100 + 50 * len(ids) and len(ids) <= 4
    # within an eps class, admission keeps arrival order
    for e in (0.1, 0.5):
        order = [i for ids, eps, _ in sorted(fr.batches, key=lambda b: b[0][0]) if e in eps
                 for i in ids]
        assert order == sorted(order)
    s = serve.summarize(reqs, srv)
    assert s["errors"] == 0 and s["latency_ms"]["p99"] >= s["latency_ms"]["p50"] > 0


def test_budget_of_one_query_serialises():
    trace = synth.poisson_requests(12, 1000.0, np.arange(5), seed=4, eps_choices=(0.5,))
    fr = FakeRunner(0.005)
    srv = _server(fr, budget=150, slots=3, max_batch=4)
    serve.run_trace(srv, trace)
    assert fr.max_live == 1 and srv.peak == 150
    assert all(len(ids) == 1 for ids, _, _ in fr.batches)


def test_budget_below_one_query_is_rejected():
    with pytest.raises(ValueError):
        _server(FakeRunner(), budget=149)


def test_runner_errors_reach_the_requests():
    def bad(batch, stream, nbytes):
        raise RuntimeError("device failure")
    srv = _server(bad, budget=1000, slots=2)
    reqs = serve.run_trace(srv, synth.poisson_requests(5, 500.0, np.arange(5), seed=5))
    assert all(r.error and "device failure" in r.error for r in reqs)
    assert serve.summarize(reqs, srv)["errors"] == 5


def test_an_empty_trace_is_empty():
    assert synth.poisson_requests(0, 1.0, np.arange(5), seed=1) == []
