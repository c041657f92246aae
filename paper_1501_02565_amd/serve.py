"""Served form: continuous batching of interpolation requests under an HBM
budget.

Requests (image pairs of mixed size and match count) arrive over time.  The
HBM budget is split evenly over the executor's slots.  When a slot is free,
waiting requests are admitted in arrival order while their device memory
(inputs, output and library workspace, ``Executor.request_bytes``) fits the
slot's share; they form one batch, launched as a single fused launch
sequence.  While a batch runs on the GPU,
new arrivals wait and are admitted into the next batch as soon as a slot and
memory free up; with several slots, batches overlap on the device.  A
request larger than the whole budget is rejected.

The scheduler (``Server``) is plain host logic with an injected clock and
executor, so it is tested on the CPU with a simulated executor.
``GpuExecutor`` runs batches through the HIP library: each slot owns an
``epic`` context (its workspace) and a HIP stream; request inputs are copied
into device buffers on admission, and flows stay on the device.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable

import numpy as np

__all__ = ["Request", "Server", "GpuExecutor", "FakeExecutor", "percentile_ms"]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                # seconds, on the server clock
    H: int
    W: int
    N: int
    K: int
    a: float = 1.0
    mode: int = 1
    cost: object = None           # host (H, W) float32
    matches: object = None        # host (N, 4) float32
    # filled by the server
    admitted: float | None = None
    done: float | None = None
    status: str = "waiting"       # waiting | running | done | rejected
    batch: int = -1
    flow: object = None           # device (H, W, 2) float32 once done

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival

    @property
    def pixels(self):
        return self.H * self.W


def percentile_ms(values, q):
    v = np.asarray([x for x in values if x is not None], dtype=np.float64)
    return float(np.percentile(v, q) * 1e3) if len(v) else float("nan")


class Server:
    """Continuous-batching scheduler.

    executor:   object with request_bytes(req), slots, submit(slot, reqs)
                and poll(slot) -> bool (True when the slot's batch is done).
    budget:     device bytes available for admitted requests.
    max_batch:  most requests in one batch.
    clock/sleep: time source (seconds) and idle wait.
    idle_s: wait between polls while work runs or waits (0 = yield and poll
    again at once).  wake_early_s: an idle server sleeps until this long
    before the next arrival and polls from there, so a sleep that overshoots
    does not delay the admission.
    """

    def __init__(self, executor, budget: int, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, idle_s: float = 50e-6,
                 wake_early_s: float = 0.0):
        self.ex = executor
        self.budget = int(budget)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.sleep = sleep
        self.idle_s = idle_s
        self.wake_early_s = wake_early_s
        self.used = 0
        self.running = {}            # slot -> list[Request]
        self.batches = 0
        self.peak_used = 0
        self.overlap_events = 0      # batches launched while another ran

    def _complete(self, slot, now):
        reqs = self.running.pop(slot)
        for r in reqs:
            r.done = now
            r.status = "done"
            self.used -= self.ex.request_bytes(r)
        self.ex.release(slot, reqs)

    @property
    def slot_budget(self):
        return self.budget // self.ex.slots

    def _form_batch(self, waiting):
        batch, need = [], 0
        free = self.slot_budget
        keep = []
        for r in waiting:
            b = self.ex.request_bytes(r)
            if b > free:
                r.status = "rejected"
                continue
            if len(batch) < self.max_batch and need + b <= free:
                batch.append(r)
                need += b
            else:
                keep.append(r)
        return batch, need, keep

    def run(self, requests, t0: float | None = None):
        """Serves `requests` (sorted by arrival, arrival relative to t0) and
        returns them with their timings filled in."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock() if t0 is None else t0
        nxt = 0
        waiting = []
        free_slots = list(range(self.ex.slots))
        while nxt < len(reqs) or waiting or self.running:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            for slot in list(self.running):
                if self.ex.poll(slot):
                    self._complete(slot, self.clock() - t0)
                    free_slots.append(slot)
            launched = False
            if waiting and free_slots:
                batch, need, waiting = self._form_batch(waiting)
                if batch:
                    slot = free_slots.pop(0)
                    now = self.clock() - t0
                    for r in batch:
                        r.admitted = now
                        r.status = "running"
                        r.batch = self.batches
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                    if self.running:
                        self.overlap_events += 1
                    self.running[slot] = batch
                    self.ex.submit(slot, batch)
                    self.batches += 1
                    launched = True
            if not launched:
                if nxt < len(reqs) and not waiting and not self.running:
                    # idle until (just before) the next arrival
                    dt = reqs[nxt].arrival - (self.clock() - t0)
                    self.sleep(dt - self.wake_early_s if dt > self.wake_early_s else self.idle_s)
                else:
                    self.sleep(self.idle_s)
        return reqs


class FakeExecutor:
    """Simulated device for host-logic tests: a batch takes
    `fixed_s + per_px_s * pixels` seconds of a simulated clock."""

    def __init__(self, clock, slots=2, fixed_s=200e-6, per_px_s=2e-9, bytes_per_px=40):
        self.clock = clock
        self.slots = slots
        self.fixed_s = fixed_s
        self.per_px_s = per_px_s
        self.bytes_per_px = bytes_per_px
        self.finish = {}
        self.log = []

    def request_bytes(self, r):
        return r.pixels * self.bytes_per_px + r.N * 200

    def submit(self, slot, reqs):
        dur = self.fixed_s + self.per_px_s * sum(r.pixels for r in reqs)
        self.finish[slot] = self.clock() + dur
        self.log.append((slot, [r.rid for r in reqs], self.clock(), self.finish[slot]))

    def poll(self, slot):
        return self.clock() >= self.finish[slot]

    def release(self, slot, reqs):
        pass


class SimClock:
    """A manual clock: sleep() advances it."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class GpuExecutor:
    """Runs batches through the HIP library.  Each slot has its own context
    (workspace of `slot_workspace` bytes) and its own stream; a batch's
    inputs are copied to device buffers when it is launched and its flows
    stay on the device."""

    def __init__(self, slots=2, slot_workspace=1 << 30, device=0, precision=0,
                 options=None):
        import torch

        import paper_1501_02565_amd as epic
        self.torch = torch
        self.epic = epic
        self.slots = slots
        self.device = torch.device("cuda", device)
        opts = dict(options or {})
        self.ctx = [epic.Context(device, slot_workspace, precision=precision, **opts)
                    for _ in range(slots)]
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.events = [None] * slots
        self.precision = precision
        self.slot_workspace = slot_workspace

    def request_bytes(self, r):
        # inputs + output on the device, plus the library workspace share
        io = 4 * r.pixels + 16 * r.N + 8 * r.pixels
        return io + self.epic.workspace_bytes(r.H, r.W, r.N, r.K, r.mode, self.precision)

    def submit(self, slot, reqs):
        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            probs = []
            for r in reqs:
                # asynchronous on the slot's stream when the host arrays are
                # pinned (pageable ones are copied before the call returns)
                c = torch.from_numpy(r.cost).to(self.device, non_blocking=True)
                m = torch.from_numpy(r.matches).to(self.device, non_blocking=True)
                r.flow = torch.empty((r.H, r.W, 2), dtype=torch.float32, device=self.device)
                probs.append((c, m, r.K, r.a, r.mode))
            self.ctx[slot].interp_batch(probs, outs=[r.flow for r in reqs], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot] = (ev, probs)

    def poll(self, slot):
        ev = self.events[slot]
        return ev is None or ev[0].query()

    def release(self, slot, reqs):
        st = [self.ctx[slot].stats(i) for i in range(len(reqs))]
        for r, s in zip(reqs, st):
            r.stats = s
        self.events[slot] = None

    def close(self):
        for c in self.ctx:
            c.close()
