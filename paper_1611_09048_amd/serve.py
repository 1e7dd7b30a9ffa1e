"""Continuous-batching render server for steering clients.

Requests arrive on the host clock; the loop admits waiting requests as slots
and memory free up, launching whatever is waiting as one batched render
(isaac_submit_batch) while earlier batches are still running on other HIP
streams, so work from successive batches overlaps on the device.  Sources
and transfer tables stay resident; each request carries its own camera,
table handles and clipping planes, so its image does not depend on what it
was batched with.  Latency runs from the request's scheduled arrival (not the
moment the loop notices it, so a busy loop cannot hide its own delay) to the
first poll that sees the request's image complete; each record also keeps when
the loop noticed the request and when it was submitted, and the executor the
host time of every submit call, so a tail can be traced to its phase.

The scheduling logic talks to an Executor; `DeviceExecutor` drives the HIP
library, `FakeExecutor` (tests) simulates completion times on a fake clock.
"""

from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Job:
    """What the executor needs to render one request."""
    rid: int
    width: int
    height: int
    direction: tuple
    tf_key: tuple                  # per source: (client, source, version) identifying its table
    tfs: list                      # control points per source
    clip: list


@dataclasses.dataclass
class Record:
    rid: int
    client: int
    arrival: float                 # scheduled arrival on the server clock
    noticed: float = math.nan      # when the loop took the request in
    submitted: float = math.nan    # when its batch's submit call returned
    done: float = math.nan         # first poll that saw its image complete
    batch: int = -1
    width: int = 0
    height: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def queued(self) -> float:
        """Arrival to submission: waiting in the loop, for a slot or for memory."""
        return self.submitted - self.arrival

    @property
    def service(self) -> float:
        """Submission to the poll that saw the image: device time plus polling delay."""
        return self.done - self.submitted


class Executor:
    def image_bytes(self, job: Job) -> int:
        return job.width * job.height * 16

    def submit(self, jobs: Sequence[Job]) -> Optional[list]:
        """Tickets, or None when admission is refused (no slot or memory)."""
        raise NotImplementedError

    def poll(self, ticket) -> bool:
        raise NotImplementedError

    def release(self, ticket) -> None:
        raise NotImplementedError


class FakeExecutor(Executor):
    """Deterministic executor for CPU tests: a batch takes `cost(jobs)` seconds on
    one of `streams` simulated streams, admission is bounded by `budget` bytes and
    `max_inflight` tickets, `fail_every` makes every n-th batch raise."""

    def __init__(self, clock, cost: Callable[[Sequence[Job]], float], budget: int, max_inflight: int = 64,
                 streams: int = 2, fail_every: int = 0):
        self.clock, self.cost, self.budget, self.max_inflight = clock, cost, budget, max_inflight
        self.stream_free = [0.0] * streams
        self.used = 0
        self.live: Dict[int, tuple] = {}
        self.next = 1
        self.batches = 0
        self.fail_every = fail_every

    def submit(self, jobs):
        need = sum(self.image_bytes(j) for j in jobs)
        if len(self.live) + len(jobs) > self.max_inflight or self.used + need > self.budget:
            return None
        self.batches += 1
        if self.fail_every and self.batches % self.fail_every == 0:
            raise RuntimeError("injected device error")
        s = int(np.argmin(self.stream_free))
        start = max(self.clock(), self.stream_free[s])
        end = start + self.cost(jobs)
        self.stream_free[s] = end
        tickets = []
        for j in jobs:
            t = self.next
            self.next += 1
            self.live[t] = (end, self.image_bytes(j))
            self.used += self.image_bytes(j)
            tickets.append(t)
        return tickets

    def poll(self, ticket):
        return self.clock() >= self.live[ticket][0]

    def release(self, ticket):
        _, b = self.live.pop(ticket)
        self.used -= b


class DeviceExecutor(Executor):
    """Renders requests of a resident volume through isaac_submit_batch."""

    def __init__(self, ctx, volume, dims, step: float = 0.5, interpolation: int = 1,
                 ert_threshold: float = 0.0, fovy_deg: float = 60.0, distance_factor: float = 2.0):
        from . import binding
        self.binding = binding
        self.ctx, self.volume, self.dims = ctx, volume, tuple(dims)
        self.step, self.interp, self.ert = step, interpolation, ert_threshold
        self.fovy, self.dist = fovy_deg, distance_factor
        self.handles: Dict[tuple, int] = {}
        self.refs: Dict[int, int] = collections.Counter()
        self.ticket_handles: Dict[int, list] = {}
        self.latest: Dict[tuple, tuple] = {}          # (client, source) -> newest table key
        self.submits = 0
        self.submit_s: List[float] = []               # host time of each submit call (tables, launch)

    def camera(self, direction):
        c = np.array(self.dims, dtype=np.float64) / 2.0
        d = np.asarray(direction, dtype=np.float64)
        d = d / np.linalg.norm(d)
        eye = c + self.dist * math.sqrt(sum(x * x for x in self.dims)) * d
        up = (0.0, 1.0, 0.0) if abs(d[0]) < 1e-12 and abs(d[1]) < 1e-12 else (0.0, 0.0, 1.0)
        return tuple(eye), tuple(c), up

    def _handle(self, key, source, points):
        h = self.handles.get(key)
        if h is None:
            h = self.ctx.set_transfer(self.volume.volume_id, source, points)
            self.handles[key] = h
        return h

    def desc(self, job: Job):
        hs = [self._handle(k, s, pts) for s, (k, pts) in enumerate(zip(job.tf_key, job.tfs))]
        eye, center, up = self.camera(job.direction)
        d = self.binding.render_desc(volume_id=self.volume.volume_id, width=job.width, height=job.height,
                                     eye=eye, center=center, up=up, fovy_deg=self.fovy, step=self.step,
                                     interpolation=self.interp, clip=job.clip, tf_handles=hs,
                                     ert_threshold=self.ert)
        return d, hs

    def submit(self, jobs):
        t0 = time.perf_counter()
        descs, hss = zip(*[self.desc(j) for j in jobs])
        for j in jobs:
            for key in j.tf_key:
                cs = key[:2]
                if cs not in self.latest or self.latest[cs][2] < key[2]:
                    self.latest[cs] = key
        tickets = self.ctx.submit_batch(list(descs))
        self.submit_s.append(time.perf_counter() - t0)
        if tickets is None:
            return None
        for t, hs in zip(tickets, hss):
            self.ticket_handles[t] = hs
            for h in hs:
                self.refs[h] += 1
        self.submits += 1
        if self.submits % 64 == 0:
            self.retire_tables(set(self.latest.values()))
        return tickets

    def poll(self, ticket):
        done, _ = self.ctx.poll(ticket)
        return done

    def image_ptr(self, ticket):
        return self.ctx.poll(ticket)[1]

    def release(self, ticket):
        self.ctx.release(ticket)
        for h in self.ticket_handles.pop(ticket, []):
            self.refs[h] -= 1

    def retire_tables(self, live_keys):
        """Release tables no client uses any more and no ticket holds (the library
        reuses a released slot only after every render reading it has finished)."""
        for key in [k for k in self.handles if k not in live_keys]:
            h = self.handles[key]
            if self.refs[h] == 0:
                self.ctx.release_transfer(h)
                del self.handles[key]


class Server:
    """The admission/batching loop (clock-agnostic)."""

    def __init__(self, executor: Executor, clock: Callable[[], float], max_batch: int = 16,
                 max_batches_in_flight: int = 3, timeout: float = math.inf,
                 on_done: Optional[Callable[[Record, object], None]] = None):
        self.ex, self.clock = executor, clock
        self.max_batch, self.max_batches = max_batch, max_batches_in_flight
        self.timeout = timeout
        self.on_done = on_done
        self.waiting: collections.deque = collections.deque()
        self.inflight: Dict[object, tuple] = {}        # ticket -> (record, batch id)
        self.batch_left: Dict[int, int] = {}
        self.records: List[Record] = []
        self.dropped: List[Record] = []
        self.failed: List[Record] = []
        self.n_batches = 0
        self.refusals = 0
        self.errors: List[str] = []

    def arrive(self, rid: int, client: int, job: Job, width: int, height: int, at: Optional[float] = None):
        """Take a request in; `at` is its scheduled arrival on the server clock (default: now)."""
        now = self.clock()
        rec = Record(rid=rid, client=client, arrival=now if at is None else at, noticed=now, width=width,
                     height=height)
        self.waiting.append((rec, job))

    def step(self) -> int:
        """One pass: retire finished work, drop timed-out waiters, launch a batch. Returns work done."""
        n = self._retire()
        now = self.clock()
        while self.waiting and now - self.waiting[0][0].arrival > self.timeout:
            rec, _ = self.waiting.popleft()
            self.dropped.append(rec)
            n += 1
        if self.waiting and len(self.batch_left) < self.max_batches:
            take = list(self.waiting)[: self.max_batch]
            while take:
                try:
                    tickets = self.ex.submit([j for _, j in take])
                except Exception as e:          # device error: fail the batch, keep serving
                    self.errors.append(str(e))
                    for _ in take:
                        rec, _j = self.waiting.popleft()
                        self.failed.append(rec)
                    return n + len(take)
                if tickets is not None:
                    break
                self.refusals += 1
                take = take[: len(take) // 2]   # admit what fits
            if take:
                bid = self.n_batches
                self.n_batches += 1
                self.batch_left[bid] = len(take)
                t_sub = self.clock()
                for t in tickets:
                    rec, _ = self.waiting.popleft()
                    rec.submitted, rec.batch = t_sub, bid
                    self.inflight[t] = (rec, bid)
                n += len(take)
        return n

    def _retire(self) -> int:
        n = 0
        for t in list(self.inflight):
            if self.ex.poll(t):
                rec, bid = self.inflight.pop(t)
                rec.done = self.clock()
                if self.on_done:
                    self.on_done(rec, t)
                self.ex.release(t)
                self.records.append(rec)
                self.batch_left[bid] -= 1
                if self.batch_left[bid] == 0:
                    del self.batch_left[bid]
                n += 1
        return n

    def idle(self) -> bool:
        return not self.waiting and not self.inflight

    def summary(self, duration: float) -> dict:
        lat = np.array([r.latency for r in self.records]) * 1e3
        out = dict(completed=len(self.records), dropped=len(self.dropped), failed=len(self.failed),
                   batches=self.n_batches, refusals=self.refusals, duration_s=duration,
                   frames_per_s=len(self.records) / duration if duration > 0 else 0.0)
        if lat.size:
            q = np.array([r.queued for r in self.records]) * 1e3
            sv = np.array([r.service for r in self.records]) * 1e3
            nd = np.array([r.noticed - r.arrival for r in self.records]) * 1e3
            out.update(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                       mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                       mean_batch=float(len(self.records) / max(1, self.n_batches)),
                       queued_ms=dict(p50=float(np.percentile(q, 50)), p99=float(np.percentile(q, 99)),
                                      max=float(q.max())),
                       service_ms=dict(p50=float(np.percentile(sv, 50)), p99=float(np.percentile(sv, 99)),
                                       max=float(sv.max())),
                       notice_delay_ms=dict(p99=float(np.percentile(nd, 99)), max=float(nd.max())))
            sub = getattr(self.ex, "submit_s", None)
            if sub:
                sub = np.array(sub) * 1e3
                out["submit_call_ms"] = dict(p50=float(np.percentile(sub, 50)), p99=float(np.percentile(sub, 99)),
                                             max=float(sub.max()))
        return out


def run(server: Server, requests, clock, sleep=time.sleep, make_job=None, drain: bool = True) -> float:
    """Feed requests at their arrival times (relative to the start) and run the loop."""
    t0 = clock()
    i = 0
    reqs = list(requests)
    while i < len(reqs) or (drain and not server.idle()):
        now = clock() - t0
        while i < len(reqs) and reqs[i].arrival <= now:
            r = reqs[i]
            server.arrive(i, r.client, make_job(i, r), r.width, r.height, at=t0 + r.arrival)
            i += 1
        worked = server.step()
        if not worked:
            nxt = reqs[i].arrival - (clock() - t0) if i < len(reqs) else 0.0
            sleep(min(max(nxt, 0.0), 2e-4) if nxt > 0 else 0.0)
    return clock() - t0


def job_from_request(rid: int, req) -> Job:
    key = tuple((req.client, s, v) for s, v in enumerate(req.tf_version))
    return Job(rid=rid, width=req.width, height=req.height, direction=req.direction, tf_key=key,
               tfs=req.tfs, clip=req.clip)
