"""The serving loop's scheduling on a fake executor and a fake clock (CPU only)."""

import math

import numpy as np
import pytest

from paper_1611_09048_amd.serve import FakeExecutor, Job, Server, job_from_request, run
from scenes import configs


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


def per_pixel_cost(jobs, ns_per_px=2.0, launch=20e-6):
    return launch + sum(j.width * j.height for j in jobs) * ns_per_px * 1e-9


def requests(rate=200.0, duration=2.0, seed=3):
    return configs.serving_requests(seed, (64, 64, 32), rate_per_client=rate / 4, duration=duration)


def test_all_requests_complete_with_consistent_latency():
    clock = FakeClock()
    ex = FakeExecutor(clock, per_pixel_cost, budget=1 << 30)
    srv = Server(ex, clock)
    reqs = requests()
    dur = run(srv, reqs, clock, sleep=clock.sleep, make_job=job_from_request)
    s = srv.summary(dur)
    assert s["completed"] == len(reqs) and s["dropped"] == 0 and s["failed"] == 0
    for r in srv.records:
        assert r.arrival <= r.submitted <= r.done
    lat = np.array([r.latency for r in srv.records])
    assert math.isclose(s["p50_ms"], np.percentile(lat, 50) * 1e3)
    assert s["p99_ms"] >= s["p50_ms"] > 0
    assert ex.used == 0 and not ex.live


def test_batches_form_under_load_and_overlap():
    clock = FakeClock()
    ex = FakeExecutor(clock, lambda jobs: 5e-3 + 1e-4 * len(jobs), budget=1 << 34, streams=2)
    srv = Server(ex, clock, max_batch=16, max_batches_in_flight=2)
    reqs = requests(rate=4000.0, duration=0.5)
    overlap = []
    orig = srv.step

    def step():
        n = orig()
        overlap.append(len(srv.batch_left))
        return n
    srv.step = step
    dur = run(srv, reqs, clock, sleep=clock.sleep, make_job=job_from_request)
    s = srv.summary(dur)
    assert s["completed"] == len(reqs)
    assert s["mean_batch"] > 2.0            # requests that arrive while others render are batched
    assert max(overlap) == 2                 # two batches in flight at once


def test_admission_respects_the_memory_budget():
    clock = FakeClock()
    peak = [0]
    budget = 3 * 1920 * 1080 * 16

    class Tracking(FakeExecutor):
        def submit(self, jobs):
            t = super().submit(jobs)
            peak[0] = max(peak[0], self.used)
            return t
    ex = Tracking(clock, per_pixel_cost, budget=budget)
    srv = Server(ex, clock, max_batch=16)
    reqs = requests(rate=2000.0, duration=0.5)
    run(srv, reqs, clock, sleep=clock.sleep, make_job=job_from_request)
    assert peak[0] <= budget
    assert srv.refusals > 0
    assert len(srv.records) == len(reqs)


def test_max_inflight_and_timeouts():
    clock = FakeClock()
    ex = FakeExecutor(clock, lambda jobs: 0.05, budget=1 << 34, max_inflight=2, streams=1)
    srv = Server(ex, clock, max_batch=8, timeout=0.02)
    reqs = requests(rate=2000.0, duration=0.2)
    run(srv, reqs, clock, sleep=clock.sleep, make_job=job_from_request)
    assert len(srv.dropped) > 0
    assert len(srv.records) + len(srv.dropped) == len(reqs)
    assert all(r.submitted - r.arrival <= 0.02 + 1e-9 for r in srv.records)


def test_device_error_fails_only_its_batch():
    clock = FakeClock()
    ex = FakeExecutor(clock, per_pixel_cost, budget=1 << 34, fail_every=3)
    srv = Server(ex, clock, max_batch=4)
    reqs = requests(rate=1000.0, duration=0.3)
    run(srv, reqs, clock, sleep=clock.sleep, make_job=job_from_request)
    assert srv.errors and len(srv.failed) > 0
    assert len(srv.records) + len(srv.failed) == len(reqs)
    assert ex.used == 0


def test_request_stream_shape():
    reqs = configs.serving_requests(5, (512, 512, 256), rate_per_client=50.0, duration=20.0)
    rate = len(reqs) / 20.0
    assert 170 < rate < 230                  # 4 clients x 50 req/s, Poisson
    kinds = {r.edit for r in reqs}
    assert kinds == {"camera", "tf", "clip"}
    assert {(r.width, r.height) for r in reqs} == set(configs.RESOLUTIONS)
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr)
    j = job_from_request(0, reqs[0])
    assert isinstance(j, Job) and len(j.tf_key) == 3


def test_latency_counts_from_the_scheduled_arrival():
    """A loop that notices a request late still counts its latency from the request's
    scheduled arrival (no coordinated omission); the phases add up."""
    clock = FakeClock()
    ex = FakeExecutor(clock, lambda jobs: 2e-3, budget=1 << 34, streams=1)
    srv = Server(ex, clock, max_batch=1, max_batches_in_flight=1)
    reqs = requests(rate=2000.0, duration=0.2)
    t0 = clock()
    run(srv, reqs, clock, sleep=clock.sleep, make_job=job_from_request)
    assert len(srv.records) == len(reqs)
    late = 0
    for r in srv.records:
        assert r.arrival == pytest.approx(t0 + reqs[r.rid].arrival, abs=1e-12)
        assert r.arrival <= r.noticed <= r.submitted <= r.done
        assert r.latency == pytest.approx(r.queued + r.service)
        late += r.noticed > r.arrival
    assert late > 0                       # the one-stream loop falls behind at this rate
    s = srv.summary(1.0)
    assert s["queued_ms"]["p99"] > s["service_ms"]["p50"]       # waiting dominates a saturated loop
    assert s["p99_ms"] >= s["queued_ms"]["p99"]
