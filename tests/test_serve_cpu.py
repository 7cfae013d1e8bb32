"""The solve server's bookkeeping on the CPU: a fake backend steps tiny
lattices with the oracle and models device time on a virtual clock.

Covered: admission by footprint, first-fit order, rejection of requests
larger than the budget, slot reuse, cancellation, fault isolation (a
non-finite request fails alone), the divergence watchdog (a diverging
request fails long before its step budget runs out), results equal to solo
runs, and the latency statistics.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_1705_11092_amd import inputs
from paper_1705_11092_amd.serve import Server, run_alone


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class FakeSlot:
    def __init__(self, req):
        wl = req.workload
        self.wl = wl
        self.fx, self.fy = oracle.force_field(wl.force_kind, wl.force_params, wl.nx, wl.ny)
        self.f = oracle.init(wl.rho, wl.ux, wl.uy, self.fx, self.fy)
        self.closed = False


class FakeBackend:
    BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f16sr": 2, "bf16sr": 2}

    def __init__(self, clock, capacity, rate=1e6):
        self.clock = clock
        self.cap = capacity
        self.rate = rate  # modelled node updates per second
        self.busy_until = 0.0
        self.opened = []
        self.advance_calls = []

    def footprint(self, req):
        return 2 * 9 * req.workload.nx * req.workload.ny * self.BYTES[req.storage]

    def capacity(self):
        return self.cap

    def open(self, req):
        s = FakeSlot(req)
        self.opened.append(s)
        return s

    def advance(self, slots, counts):
        self.advance_calls.append(list(counts))
        work = 0
        for s, c in zip(slots, counts):
            if c:
                s.f = oracle.run(s.f, s.fx, s.fy, s.wl.s, c, bc_y=s.wl.bc_y, nthreads=1)
            work += c * s.wl.nx * s.wl.ny
        self.busy_until = max(self.busy_until, self.clock.now()) + work / self.rate

    def finish(self, slot):
        return oracle.moments(slot.f, slot.fx, slot.fy)

    def watch(self, slot):
        rho, ux, uy = oracle.moments(slot.f, slot.fx, slot.fy)
        return (float(rho.sum()), float((rho * ux).sum()), float((rho * uy).sum()))

    def watched(self, token):
        return token

    def fence(self):
        return self.busy_until

    def wait(self, ev):
        self.clock.sleep_until(ev)

    def collect(self, pending):
        return pending

    def close(self, slot):
        assert not slot.closed
        slot.closed = True


def _stream(count=12, seed=4, rate=50.0, n_lo=8, n_hi=24, steps_lo=20, steps_hi=200):
    return inputs.served_stream(count=count, seed=seed, rate=rate, n_lo=n_lo, n_hi=n_hi,
                                steps_lo=steps_lo, steps_hi=steps_hi)


def test_all_requests_complete_and_match_solo_runs():
    reqs = _stream()
    clock = VirtualClock()
    be = FakeBackend(clock, capacity=10**9)
    rep = Server(be, clock=clock, min_tick=8, max_tick=64).run(reqs)
    assert all(r.status == "done" for r in rep.results.values())
    assert all(s.closed for s in be.opened)
    for req in reqs[:5]:
        clock2 = VirtualClock()
        solo = run_alone(FakeBackend(clock2, capacity=10**9), req)
        got = rep.results[req.rid]
        assert np.array_equal(got.ux, solo.ux) and np.array_equal(got.rho, solo.rho)
    # Served LUPs are exactly sum N^2 * steps.
    assert rep.lups == sum(r.workload.nx * r.workload.ny * r.workload.steps for r in reqs)
    s = rep.summary()
    assert s["done"] == len(reqs)
    lat = rep.latencies()
    assert s["p50_latency_s"] == pytest.approx(float(np.percentile(lat, 50)))
    assert s["p99_latency_s"] == pytest.approx(float(np.percentile(lat, 99)))
    for r in rep.results.values():
        assert r.finished >= r.admitted >= r.arrival


def test_admission_respects_the_budget():
    reqs = _stream(count=10, n_lo=16, n_hi=16)
    clock = VirtualClock()
    fp = 2 * 9 * 16 * 16 * 4
    be = FakeBackend(clock, capacity=2 * fp + fp // 2)
    for r in reqs:
        r.storage = "f32"
    rep = Server(be, clock=clock, min_tick=8, max_tick=64).run(reqs)
    assert rep.max_active <= 2
    assert rep.peak_bytes <= be.cap
    assert all(r.status == "done" for r in rep.results.values())


def test_too_large_requests_are_rejected_others_served():
    reqs = _stream(count=6)
    big = dataclasses.replace(reqs[0], rid=99, workload=inputs.kolmogorov(200, 1e-6, 1, 0.8, 10))
    clock = VirtualClock()
    be = FakeBackend(clock, capacity=2 * 9 * 64 * 64 * 4)
    rep = Server(be, clock=clock).run(reqs + [big])
    assert rep.results[99].status == "rejected"
    assert sum(r.status == "done" for r in rep.results.values()) == len(reqs)


def test_first_fit_lets_small_requests_pass_a_blocked_large_one():
    big = inputs.Request(1, 0.0, inputs.kolmogorov(40, 1e-6, 1, 0.8, 400), "f32")
    big2 = inputs.Request(2, 0.001, inputs.kolmogorov(40, 1e-6, 1, 0.8, 100), "f32")
    small = inputs.Request(3, 0.002, inputs.kolmogorov(8, 1e-6, 1, 0.8, 50), "f32")
    clock = VirtualClock()
    fp40 = 2 * 9 * 40 * 40 * 4
    be = FakeBackend(clock, capacity=fp40 + 2 * 9 * 8 * 8 * 4)
    rep = Server(be, clock=clock, min_tick=8, max_tick=16).run([big, big2, small])
    r = rep.results
    assert all(x.status == "done" for x in r.values())
    assert r[3].admitted < r[2].admitted  # the small one did not wait for big2


def test_cancellation_frees_the_slot():
    reqs = _stream(count=8)
    clock = VirtualClock()
    be = FakeBackend(clock, capacity=10**9)
    srv = Server(be, clock=clock, min_tick=8, max_tick=16)
    srv.cancel(reqs[0].rid)
    srv.cancel(reqs[3].rid)
    rep = srv.run(reqs)
    assert rep.results[reqs[0].rid].status == "cancelled"
    assert rep.results[reqs[3].rid].status == "cancelled"
    assert sum(r.status == "done" for r in rep.results.values()) == len(reqs) - 2
    assert all(s.closed for s in be.opened)


def test_a_nonfinite_request_fails_alone():
    reqs = _stream(count=6)
    bad = reqs[2]
    bad.workload.rho = bad.workload.rho.copy()
    bad.workload.rho[1, 1] = math.nan
    clock = VirtualClock()
    be = FakeBackend(clock, capacity=10**9)
    rep = Server(be, clock=clock, min_tick=8, max_tick=32).run(reqs)
    assert rep.results[bad.rid].status == "failed"
    others = [r for r in rep.results.values() if r.rid != bad.rid]
    assert all(r.status == "done" and all(math.isfinite(v) for v in r.totals) for r in others)
    # And the others are unchanged by the failing neighbour.
    req = reqs[0]
    solo = run_alone(FakeBackend(VirtualClock(), capacity=10**9), req)
    assert np.array_equal(rep.results[req.rid].ux, solo.ux)


def test_watchdog_stops_a_diverging_request_early():
    # A request whose state is NaN from the start and whose step budget is
    # 200,000 steps: the watchdog (every 4 ticks of at most 16 steps) fails
    # it within its first 64 + 16 steps and frees its slot; the others finish
    # and equal their solo runs.
    reqs = _stream(count=6)
    bad = dataclasses.replace(reqs[1], workload=dataclasses.replace(reqs[1].workload, steps=200_000))
    bad.workload.rho = bad.workload.rho.copy()
    bad.workload.rho[2, 3] = math.nan
    reqs[1] = bad
    clock = VirtualClock()
    be = FakeBackend(clock, capacity=10**9)
    rep = Server(be, clock=clock, min_tick=8, max_tick=16, watch_every=4).run(reqs)
    r = rep.results[bad.rid]
    assert r.status == "failed" and "watchdog" in r.message, r.message
    nodes = bad.workload.nx * bad.workload.ny
    others = sum(q.workload.nx * q.workload.ny * q.workload.steps for q in reqs if q.rid != bad.rid)
    assert rep.lups - others <= (4 * 16 + 16) * nodes
    for q in reqs:
        if q.rid == bad.rid:
            continue
        assert rep.results[q.rid].status == "done"
        solo = run_alone(FakeBackend(VirtualClock(), capacity=10**9), q)
        assert np.array_equal(rep.results[q.rid].ux, solo.ux)
    assert all(s.closed for s in be.opened)
    # With the watchdog off the same request runs out its budget first.
    clock = VirtualClock()
    be = FakeBackend(clock, capacity=10**9)
    rep = Server(be, clock=clock, min_tick=8, max_tick=16, watch_every=0).run(
        [dataclasses.replace(bad, workload=dataclasses.replace(bad.workload, steps=400))])
    assert rep.results[bad.rid].status == "failed"
    assert rep.lups == 400 * nodes


def test_tick_length_is_a_bounded_power_of_two():
    srv = Server(FakeBackend(VirtualClock(), 1, rate=6e10), min_tick=32, max_tick=4096, tick_s=0.02)
    for nodes in (1, 100, 10**4, 10**6, 10**7, 10**9):
        k = srv._tick_steps(nodes)
        assert 32 <= k <= 4096 and (k & (k - 1)) == 0


def test_served_stream_recipe_is_seeded_and_in_range():
    a = inputs.served_stream(count=50, seed=1)
    b = inputs.served_stream(count=50, seed=1)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    for r in a:
        assert 64 <= r.workload.nx <= 2048 and r.workload.nx == r.workload.ny
        assert 1000 <= r.workload.steps <= 100000
        assert r.storage in ("f32", "f16sr")
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
