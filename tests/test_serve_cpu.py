"""The serving loop's state machine on the CPU, with an oracle-backed fake
engine and a simulated clock: FIFO admission by footprint, the heap budget is
never exceeded, oversize requests are rejected, every result reaches its own
request, latencies and nearest-rank percentiles are consistent."""
import numpy as np
import pytest

from oracle.pyoracle import Oracle
from paper_2105_10576_amd import cases
from paper_2105_10576_amd.serve import Server, nearest_rank


class FakeEngine:
    def __init__(self, heap, max_slots, footprint, clock):
        self.heap, self.max_slots, self.fp, self.clock = heap, max_slots, footprint, clock
        self.slots = {}
        self.used = 0

    def admit(self, case):
        need = self.fp(case)
        if len(self.slots) >= self.max_slots or self.used + need > self.heap:
            return None
        o = Oracle(case)
        o.viscous_step(case["dt_vd"])
        rc, kf, E = o.capillary_relax(case["dt_vd"], case["n_sub"], case["max_iters"], case["tol"])
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = dict(left=1 + kf, kf=kf, need=need, alpha=o.get("alpha"), p=o.get("p"), U=o.get("U"))
        self.used += need
        return slot

    def run(self, ticks):
        for _ in range(ticks):
            self.clock[0] += 1e-3
            for s in self.slots.values():
                if s["left"] > 0:
                    s["left"] -= 1

    def poll(self):
        done = [k for k, s in self.slots.items() if s["left"] == 0]
        return done, len(self.slots) - len(done)

    def fetch(self, slot):
        s = self.slots[slot]
        return dict(alpha=s["alpha"], p=s["p"], U=s["U"], k_f=s["kf"], status=0)

    def release(self, slot):
        self.used -= self.slots.pop(slot)["need"]

    def free(self):
        return self.heap - self.used, self.max_slots - len(self.slots)


def _requests(n):
    reqs = []
    for r in range(n):
        c = cases.channel_bubble(nx=32 + 16 * (r % 3), ny=8 + 8 * (r % 2), n_sub=12, max_iters=2 + r % 3)
        reqs.append(c)
    return reqs


def test_fifo_budget_and_results():
    clock = [0.0]
    fp = lambda c: int(c["nx"]) * int(c["ny"]) * 1000
    reqs = _requests(8)
    heap = 2 * 64 * 16 * 1000          # room for about two of the largest requests
    eng = FakeEngine(heap, 3, fp, clock)
    arrivals = [0.0005 * i for i in range(len(reqs))]

    def sleep(dt):
        clock[0] += dt

    srv = Server(eng, fp, clock=lambda: clock[0], sleep=sleep, heap_bytes=heap)
    res, summ = srv.run(reqs, arrivals, keep_fields=True)
    assert summ["served"] == 8 and summ["rejected"] == 0
    assert summ["admit_order"] == sorted(summ["admit_order"])      # first come, first served
    assert summ["peak_resident_bytes"] <= heap
    for r in res:
        o = Oracle(reqs[r["request"]])
        o.viscous_step(reqs[r["request"]]["dt_vd"])
        c = reqs[r["request"]]
        o.capillary_relax(c["dt_vd"], c["n_sub"], c["max_iters"], c["tol"])
        assert np.array_equal(r["alpha"], o.get("alpha"))
        assert r["latency"] >= 0 and r["done"] >= r["admitted"] >= r["arrival"]
    lat = sorted(r["latency"] for r in res)
    assert summ["p50_latency_s"] == lat[3] and summ["p99_latency_s"] == lat[-1]


def test_oversize_request_is_rejected():
    clock = [0.0]
    fp = lambda c: int(c["nx"]) * int(c["ny"]) * 1000
    reqs = _requests(3)
    eng = FakeEngine(10, 2, fp, clock)
    srv = Server(eng, fp, clock=lambda: clock[0], sleep=lambda dt: None, heap_bytes=10)
    res, summ = srv.run(reqs, [0.0, 0.0, 0.0])
    assert summ["rejected"] == 3 and all(r["rejected"] for r in res)


def test_nearest_rank():
    v = list(range(1, 65))
    assert nearest_rank(v, 50) == 32 and nearest_rank(v, 99) == 64 and nearest_rank(v, 100) == 64
    assert nearest_rank([5.0], 99) == 5.0
