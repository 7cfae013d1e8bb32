"""Continuous-batching solve server for lattice Boltzmann requests.

Requests (a lattice workload, a step count and a storage type) arrive over
time.  The server admits a waiting request as soon as its HBM footprint
(both population buffers) fits in the budget, keeps the populations of every
admitted request resident on the device, and advances all admitted requests
together: each tick is one batched launch sequence in which request j takes
min(K, steps left) steps.  A request that completes in a tick has its
density and velocity fields copied to the host behind the tick's kernels;
the server launches the next tick before it waits for those copies, so host
bookkeeping overlaps device work.  Latency is measured from arrival to the
moment the result is on the host.

The batched kernel updates every node with exactly the arithmetic of a
single-lattice step, so a request's result does not depend on what else
was in the batch.

A watchdog guards against the method's one failure mode, divergence (an
unstable choice of rates, Sec. IV C): every ``watch_every`` ticks the
server has the FP64 mass and momentum of every active request reduced on
the device behind the tick, and a request whose totals are NaN or Inf is
failed and its slot freed at once, instead of running out its step budget.

The server is backend-agnostic: ``GpuBackend`` drives the HIP library; a
test backend can model time instead.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import inputs


# ---------------------------------------------------------------------------
# Clocks
# ---------------------------------------------------------------------------

class WallClock:
    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(min(d, 0.05))


# ---------------------------------------------------------------------------
# Records
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    rid: int
    status: str  # "done" | "failed" | "rejected" | "cancelled"
    steps: int = 0
    nodes: int = 0
    arrival: float = 0.0
    admitted: float = math.nan
    finished: float = math.nan
    rho: Optional[np.ndarray] = None
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None
    totals: Optional[tuple] = None
    message: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def queue_delay(self) -> float:
        return self.admitted - self.arrival


@dataclasses.dataclass
class Report:
    results: Dict[int, Result]
    makespan: float
    lups: float
    ticks: int
    max_active: int
    peak_bytes: int

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results.values() if r.status == "done"])

    def summary(self) -> dict:
        lat = self.latencies()
        done = len(lat)
        return {
            "requests": len(self.results),
            "done": done,
            "failed": sum(r.status == "failed" for r in self.results.values()),
            "rejected": sum(r.status == "rejected" for r in self.results.values()),
            "cancelled": sum(r.status == "cancelled" for r in self.results.values()),
            "p50_latency_s": float(np.percentile(lat, 50)) if done else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if done else None,
            "mean_queue_delay_s": float(np.mean([r.queue_delay for r in self.results.values()
                                                 if r.status == "done"])) if done else None,
            "makespan_s": self.makespan,
            "mlups": self.lups / self.makespan / 1e6 if self.makespan > 0 else None,
            "ticks": self.ticks,
            "max_active": self.max_active,
            "peak_resident_bytes": self.peak_bytes,
        }


# ---------------------------------------------------------------------------
# GPU backend
# ---------------------------------------------------------------------------

class _Pending:
    """Result of one request whose device-to-host copies are in flight."""

    def __init__(self, slot, host):
        self.slot = slot
        self.host = host


class GpuBackend:
    """Backend on the HIP library: one clbm.Lattice per request, advanced
    together by a clbm.Batch rebuilt whenever the set of requests changes.
    With inplace=True every request streams in place (one buffer instead of
    two): half the footprint, so twice the requests fit a budget, with
    bitwise the same results."""

    def __init__(self, budget_bytes: Optional[int] = None, budget_frac: float = 0.8,
                 device: str = "cuda", autotune_cache: Optional[str] = None,
                 rate_lups: float = 6e10, inplace: bool = False):
        import torch

        from . import clbm
        self.torch, self.clbm = torch, clbm
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(free * budget_frac)
        self.budget = int(budget_bytes)
        self.autotune_cache = autotune_cache
        self.rate = rate_lups  # for choosing the tick length
        self.inplace = bool(inplace)
        self._batch = None
        self._members: tuple = ()

    def footprint(self, req) -> int:
        wl = req.workload
        return (1 if self.inplace else 2) * self.clbm.buffer_bytes(wl.nx, wl.ny, req.storage)

    def capacity(self) -> int:
        return self.budget

    def open(self, req):
        return self.clbm.lattice_from_workload(req.workload, storage=req.storage,
                                               device=str(self.device), stream=self.stream,
                                               inplace=self.inplace)

    def _ensure_batch(self, slots):
        key = tuple(id(s) for s in slots)
        if key != self._members:
            if self._batch is not None:
                self._batch.close()
            self._batch = self.clbm.Batch(slots, stream=self.stream)
            if self.autotune_cache:
                self._batch.autotune(self.autotune_cache)
            self._members = key
        return self._batch

    def advance(self, slots, counts):
        self._ensure_batch(slots).step_each(counts)

    def finish(self, slot) -> _Pending:
        torch = self.torch
        rho, ux, uy, _ = slot.moments(fields=True, totals=False)
        host = []
        for t in (rho, ux, uy):
            h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
            h.copy_(t, non_blocking=True)
            host.append(h)
        return _Pending(slot, host)

    def watch(self, slot):
        """Enqueue the FP64 totals {mass, momentum} of a request's state
        (clbm_moments_noalloc: no allocation in the library, no wait) and
        their copy to pinned host memory; read them with watched() once a
        later fence has passed."""
        torch = self.torch
        dev = torch.empty(3, dtype=torch.float64, device=self.device)
        slot.moments_noalloc(totals=dev)
        host = torch.empty(3, dtype=torch.float64, pin_memory=True)
        host.copy_(dev, non_blocking=True)
        return host

    def watched(self, token):
        return tuple(float(v) for v in token.numpy())

    def fence(self):
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, ev):
        ev.synchronize()

    def collect(self, pending: _Pending):
        rho, ux, uy = (h.numpy() for h in pending.host)
        return rho, ux, uy

    def close(self, slot):
        if self._batch is not None and id(slot) in self._members:
            self._batch.close()
            self._batch = None
            self._members = ()
        slot.close()

    def shutdown(self):
        if self._batch is not None:
            self._batch.close()
            self._batch = None


# ---------------------------------------------------------------------------
# Server
# ---------------------------------------------------------------------------

class Server:
    """Admit, batch and complete requests as they arrive (see module doc)."""

    def __init__(self, backend, clock=None, max_active: int = 1024, tick_s: float = 0.02,
                 min_tick: int = 32, max_tick: int = 4096, log=None, watch_every: int = 8):
        self.backend = backend
        self.clock = clock or WallClock()
        self.max_active = max_active
        self.tick_s = tick_s
        self.min_tick, self.max_tick = min_tick, max_tick
        self.log = log
        # Watchdog period in ticks (0: off; the final fields are checked
        # either way).
        self.watch_every = watch_every
        self._cancel = set()

    def cancel(self, rid: int):
        self._cancel.add(rid)

    def _tick_steps(self, active_nodes: int) -> int:
        rate = getattr(self.backend, "rate", 6e10)
        k = int(self.tick_s * rate / max(active_nodes, 1))
        k = max(self.min_tick, min(self.max_tick, k))
        return 1 << (k.bit_length() - 1)  # power of two: stable graph shapes

    def run(self, requests: List[inputs.Request]) -> Report:
        be = self.backend
        clock = self.clock
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: List[inputs.Request] = []
        active: Dict[int, list] = {}  # rid -> [req, slot, remaining, footprint]
        results: Dict[int, Result] = {}
        used = peak = 0
        lups = 0.0
        ticks = max_act = 0
        inflight = None  # (event, [(rid, pending, footprint, slot)], [(rid, watch token)])
        watch = self.watch_every > 0 and hasattr(be, "watch")
        t0 = clock.now()

        def now():
            return clock.now() - t0

        def finalize(batch):
            nonlocal used
            ev, items, watched = batch
            be.wait(ev)
            t = now()
            # Watchdog: fail a still active request whose totals diverged.
            for rid, token in watched:
                if rid not in active:
                    continue
                tot = be.watched(token)
                if not all(math.isfinite(v) for v in tot):
                    req, slot, left, fp = active.pop(rid)
                    r = results[rid]
                    r.status, r.finished, r.totals = "failed", t, tot
                    r.message = (f"diverged: non-finite mass or momentum within its first "
                                 f"{req.workload.steps - left} of {req.workload.steps} steps (watchdog)")
                    be.close(slot)
                    used -= fp
            for rid, pend, fp, slot in items:
                rho, ux, uy = be.collect(pend)
                r = results[rid]
                r.finished = t
                r.rho, r.ux, r.uy = rho, ux, uy
                tot = (float(np.sum(rho)), float(np.sum(rho * ux)), float(np.sum(rho * uy)))
                r.totals = tot
                if not all(math.isfinite(v) for v in tot):
                    r.status, r.message = "failed", "non-finite mass or momentum"
                else:
                    r.status = "done"
                be.close(slot)
                used -= fp

        while pending or waiting or active or inflight:
            tnow = now()
            while pending and pending[0].arrival <= tnow:
                req = pending.popleft()
                waiting.append(req)
                results[req.rid] = Result(req.rid, "waiting", steps=req.workload.steps,
                                          nodes=req.workload.nx * req.workload.ny,
                                          arrival=req.arrival)
            # Cancellations of waiting and active requests.
            for req in [w for w in waiting if w.rid in self._cancel]:
                waiting.remove(req)
                results[req.rid].status = "cancelled"
            for rid in [k for k in active if k in self._cancel]:
                _, slot, _, fp = active.pop(rid)
                be.close(slot)
                used -= fp
                results[rid].status = "cancelled"
            # Admission, first fit in arrival order.
            for req in list(waiting):
                fp = be.footprint(req)
                if fp > be.capacity():
                    waiting.remove(req)
                    results[req.rid].status = "rejected"
                    results[req.rid].message = "larger than the HBM budget"
                    continue
                if used + fp <= be.capacity() and len(active) < self.max_active:
                    waiting.remove(req)
                    try:
                        slot = be.open(req)
                    except Exception as exc:  # resource failure: report, keep serving
                        results[req.rid].status = "failed"
                        results[req.rid].message = f"open failed: {exc}"
                        continue
                    used += fp
                    peak = max(peak, used)
                    active[req.rid] = [req, slot, req.workload.steps, fp]
                    results[req.rid].admitted = now()
            if active:
                nodes = sum(a[0].workload.nx * a[0].workload.ny for a in active.values())
                K = self._tick_steps(nodes)
                rids = list(active)
                counts = [min(K, active[r][2]) for r in rids]
                be.advance([active[r][1] for r in rids], counts)
                ticks += 1
                max_act = max(max_act, len(rids))
                done_items = []
                for r, c in zip(rids, counts):
                    a = active[r]
                    a[2] -= c
                    lups += c * a[0].workload.nx * a[0].workload.ny
                    if a[2] == 0:
                        done_items.append((r, be.finish(a[1]), a[3], a[1]))
                        del active[r]
                watched = []
                if watch and ticks % self.watch_every == 0:
                    watched = [(r, be.watch(active[r][1])) for r in active]
                ev = be.fence()
                if inflight is not None:
                    finalize(inflight)
                inflight = (ev, done_items, watched)
            elif inflight is not None:
                finalize(inflight)
                inflight = None
            elif pending and not waiting:
                clock.sleep_until(t0 + pending[0].arrival)
            elif waiting and not active:
                # Nothing fits and nothing runs: only possible if capacity
                # shrank; reject the rest rather than spin.
                for req in waiting:
                    results[req.rid].status = "rejected"
                    results[req.rid].message = "no capacity"
                waiting.clear()
        be_shutdown = getattr(be, "shutdown", None)
        if be_shutdown:
            be_shutdown()
        return Report(results, now(), lups, ticks, max_act, peak)


def run_alone(backend, req) -> Result:
    """The same request through the server on its own (arrival at t = 0)."""
    solo = dataclasses.replace(req, arrival=0.0)
    rep = Server(backend).run([solo])
    return rep.results[req.rid]
