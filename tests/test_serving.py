"""CPU checks of the serving layer: the seeded request stream, the FIFO
admission loop under an HBM budget (driven by a simulated device), the
latency summary, and the group C-ABI's argument checks (no GPU call)."""
import ctypes
import math
import os

import numpy as np
import pytest

from paper_2403_15773_amd import serve, tslb


def test_request_stream_matches_its_recipe():
    reqs = serve.make_requests(256, rate=20.0, master_seed=5)
    again = serve.make_requests(256, rate=20.0, master_seed=5)
    assert [vars(a) for a in reqs] == [vars(b) for b in again]  # seeded
    t = np.array([r.arrival for r in reqs])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    # exponential gaps of mean 1/20 s: the mean of 255 gaps has std 3.1 ms
    assert abs(gaps.mean() - 0.05) < 0.012
    # exponential: the std equals the mean (within sampling error)
    assert 0.7 < gaps.std() / gaps.mean() < 1.3
    Ls = [r.L for r in reqs]
    assert set(Ls) == set(serve.SIZES)
    assert 0.35 < sum(r.setup == "jet" for r in reqs) / 256 < 0.65
    assert all(500 <= r.re <= 5000 and 10 <= r.we <= 2000 for r in reqs)
    assert all(500 <= r.steps <= 5000 for r in reqs)
    # log-uniform: the median of log Re sits near the middle of [log 500, log 5000]
    mid = 0.5 * (math.log(500) + math.log(5000))
    assert abs(np.median([math.log(r.re) for r in reqs]) - mid) < 0.3
    # different master seeds give different streams
    other = serve.make_requests(16, master_seed=6)
    assert [r.L for r in other] != Ls[:16] or [r.steps for r in other] != [r.steps for r in reqs[:16]]


def test_request_setup_follows_the_recipe():
    jet = serve.Request(0, 0.0, 64, "jet", 1000.0, 100.0, 600, 123)
    p, f = serve.request_setup(jet)
    assert (p["nx"], p["ny"], p["nz"]) == (64, 64, 64)
    assert p["bc"] == (1, 1, 1, 1, 2, 3) and p["inlet_d"] == 8.0 and p["inlet_u"] == 0.05
    assert math.isclose(p["nu"], 0.05 * 8 / 1000) and math.isclose(p["sigma"], 0.05 ** 2 * 8 / 100)
    assert f["phi"].shape == (64, 64, 64) and f["phi"].dtype == np.float32 and not f["phi"].any()
    drop = serve.Request(1, 0.0, 32, "droplet", 500.0, 20.0, 600, 7)
    p, f = serve.request_setup(drop)
    assert p["bc"] == (0,) * 6
    assert math.isclose(p["nu"], 0.05 * 16 / 500) and math.isclose(p["sigma"], 0.05 ** 2 * 16 / 20)
    assert f["phi"][16, 16, 16] > 0.99 and f["phi"][0, 0, 0] < 1e-5
    assert 0 < np.abs(f["u"]).max() <= 1e-3
    assert serve.request_setup_params_only(drop)[0] == p


class FakeDevice:
    """A device model: every poll advances each member by one step and costs
    `per_poll` seconds plus `per_node` per member node of simulated time."""

    def __init__(self, clock, per_poll=1e-4, per_node=2e-9, bytes_per_node=88):
        self.clock = clock
        self.per_poll, self.per_node, self.bpn = per_poll, per_node, bytes_per_node
        self.members = {}
        self.order = []
        self.peak_bytes = 0
        self.next_key = 0

    def prepare(self, req):
        return req.L

    def required_bytes(self, req):
        return self.bpn * req.L ** 3

    def create(self, req, prepared):
        self.next_key += 1
        return {"key": self.next_key, "req": req, "left": None, "done": 0}

    def admit(self, h, nsteps):
        h["left"] = nsteps
        self.members[h["key"]] = h
        self.order.append(h["req"].id)
        self.peak_bytes = max(self.peak_bytes, sum(self.required_bytes(m["req"]) for m in self.members.values()))
        return True

    def key(self, h):
        return h["key"]

    def poll(self):
        out = [m for m in self.members.values() if m["left"] == 0]
        for m in out:
            del self.members[m["key"]]
        work = sum(m["req"].L ** 3 for m in self.members.values() if m["left"] > 0)
        for m in self.members.values():
            if m["left"] > 0:
                m["left"] -= 1
                m["done"] += 1
        self.clock.t += self.per_poll + self.per_node * work
        return out

    def finish(self, h):
        return {"finite": True, "steps_done": h["done"]}


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def test_serving_loop_fifo_budget_and_summary():
    reqs = serve.make_requests(40, rate=50.0, master_seed=11, sizes=(32, 48, 64), steps=(20, 80))
    clock = FakeClock()
    dev = FakeDevice(clock)
    budget = 88 * (64 ** 3 + 48 ** 3)  # room for about two mid-size requests
    recs = serve.serve(reqs, dev, budget, max_domains=3, clock=clock, sleep=clock.sleep, prepare_workers=2)
    assert dev.peak_bytes <= budget
    # FIFO: admission order is arrival order, and admission times never decrease
    assert dev.order == [r.id for r in sorted(reqs, key=lambda r: r.arrival)]
    adm = [rec.admitted for rec in sorted(recs, key=lambda x: x.req.arrival)]
    assert all(b >= a for a, b in zip(adm, adm[1:]))
    for rec in recs:
        assert rec.extra["steps_done"] == rec.req.steps
        assert rec.req.arrival <= rec.admitted <= rec.done
    s = serve.summarise(recs)
    lat = sorted(r.latency for r in recs)
    assert s["requests"] == 40 and s["unstable"] == 0
    assert math.isclose(s["p50_latency_s"], float(np.percentile(lat, 50)))
    assert lat[0] <= s["p50_latency_s"] <= s["p99_latency_s"] <= lat[-1]
    assert math.isclose(s["aggregate_glups"] * 1e9 * s["makespan_s"], sum(r.L ** 3 * r.steps for r in reqs))


def test_serving_loop_never_exceeds_the_slot_count():
    reqs = serve.make_requests(12, rate=1000.0, master_seed=3, sizes=(32,), steps=(5, 10))
    clock = FakeClock()

    class Counting(FakeDevice):
        peak = 0

        def admit(self, h, n):
            ok = super().admit(h, n)
            Counting.peak = max(Counting.peak, len(self.members))
            return ok

    dev = Counting(clock)
    recs = serve.serve(reqs, dev, 10 ** 12, max_domains=2, clock=clock, sleep=clock.sleep)
    assert Counting.peak <= 2 and all(not math.isnan(r.done) for r in recs)


def test_request_larger_than_the_budget_is_an_error():
    """A request that could never fit (even on an empty device) fails instead of
    blocking the queue for ever."""
    reqs = serve.make_requests(3, rate=100.0, master_seed=2, sizes=(48,), steps=(5, 6))
    clock = FakeClock()
    with pytest.raises(ValueError, match="more than the budget"):
        serve.serve(reqs, FakeDevice(clock), 88 * 32 ** 3, max_domains=4, clock=clock, sleep=clock.sleep)


def test_refused_lattice_keeps_its_place():
    """A lattice the device refuses once is offered again after the next poll,
    before any lattice whose creation started later."""
    reqs = serve.make_requests(10, rate=1000.0, master_seed=4, sizes=(32,), steps=(5, 10))
    clock = FakeClock()

    class RefusesOnce(FakeDevice):
        refused = []

        def admit(self, h, n):
            rid = h["req"].id
            if rid == 3 and not RefusesOnce.refused:
                RefusesOnce.refused.append(rid)
                return False
            return super().admit(h, n)

    dev = RefusesOnce(clock)
    recs = serve.serve(reqs, dev, 10 ** 12, max_domains=4, clock=clock, sleep=clock.sleep, prepare_workers=2)
    assert RefusesOnce.refused == [3]
    assert dev.order == [r.id for r in sorted(reqs, key=lambda r: r.arrival)]
    assert all(rec.extra["steps_done"] == rec.req.steps for rec in recs)


def test_budget_defaults_to_the_backends_free_memory():
    reqs = serve.make_requests(6, rate=100.0, master_seed=9, sizes=(32, 48), steps=(5, 8))
    clock = FakeClock()

    class Sized(FakeDevice):
        def admission_budget(self):
            return 88 * 48 ** 3  # one request at a time

    dev = Sized(clock)
    serve.serve(reqs, dev, None, max_domains=4, clock=clock, sleep=clock.sleep)
    assert 0 < dev.peak_bytes <= 88 * 48 ** 3


def test_summary_reports_offered_load_and_busy_fraction():
    reqs = serve.make_requests(20, rate=50.0, master_seed=11, sizes=(32,), steps=(20, 40))
    clock = FakeClock()
    recs = serve.serve(reqs, FakeDevice(clock), 10 ** 12, max_domains=8, clock=clock, sleep=clock.sleep)
    s = serve.summarise(recs, busy_s=0.5 * (max(r.done for r in recs) - reqs[0].arrival))
    assert math.isclose(s["device_busy_frac"], 0.5)
    span_arrivals = max(r.arrival for r in reqs) - min(r.arrival for r in reqs)
    assert math.isclose(s["offered_glups"] * 1e9 * span_arrivals, sum(r.L ** 3 * r.steps for r in reqs))
    assert serve.summarise(recs)["device_busy_frac"] is None


# ---- the group C-ABI: argument checks only (no device is touched) ----

@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tslb.LIB_PATH):
        from paper_2403_15773_amd import build
        build.build()
    return tslb.load_library()


def test_group_create_rejects_bad_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.tslb_group_create(1 << 20, 4, None, None) == tslb.E_INVAL
    assert lib.tslb_group_create(1 << 20, 0, None, ctypes.byref(h)) == tslb.E_INVAL
    assert b"max_domains" in lib.tslb_group_last_error(None)
    assert lib.tslb_group_create(1 << 20, 5000, None, ctypes.byref(h)) == tslb.E_INVAL
    assert lib.tslb_group_create(0, 4, None, ctypes.byref(h)) == tslb.E_INVAL
    assert h.value is None


def test_group_calls_reject_null_handles(lib):
    n = ctypes.c_int32(7)
    assert lib.tslb_group_admit(None, None, 1) == tslb.E_INVAL
    assert lib.tslb_group_poll(None, None, 0, ctypes.byref(n)) == tslb.E_INVAL
    assert lib.tslb_group_status(None, None, None, None) == tslb.E_INVAL
    lib.tslb_group_destroy(None)  # no-op
    assert b"group is NULL" in lib.tslb_group_last_error(None)
