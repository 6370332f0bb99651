"""Request loop of the relaxation service: continuous batching on one GPU.

Requests (case dictionaries from cases.py: one viscous-drag step plus one
capillary relaxation each) arrive at given times.  The loop admits the head
of the arrival queue whenever the engine has a free slot and a heap region
that fits the request's workspace footprint (first come, first served: the
head waits rather than being overtaken), advances every resident request by
one tick, fetches and releases finished requests, and records each request's
latency from arrival to results on the host.

The engine is any object with admit(case) -> slot | None, run(ticks),
poll() -> (done_slots, n_active), fetch(slot) -> dict, release(slot) and
free() -> (largest_region, free_slots); oscar.Engine is the GPU one.
"""
from __future__ import annotations

import time


def nearest_rank(values, q):
    """q-th percentile by nearest rank (q in (0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, int(-(-q * len(v) // 100)))   # ceil(q n / 100)
    return v[k - 1]


class Server:
    def __init__(self, engine, footprint, clock=time.perf_counter, sleep=time.sleep, heap_bytes=None):
        """footprint(case) -> bytes a request occupies in the engine heap;
        heap_bytes: total heap (requests larger than it are rejected)."""
        self.engine = engine
        self.footprint = footprint
        self.clock = clock
        self.sleep = sleep
        self.heap_bytes = heap_bytes

    def run(self, requests, arrivals, keep_fields=False, max_wall=None, progress=None, progress_every=25):
        """Serve `requests` arriving at times `arrivals` (seconds after the
        start, non-decreasing).  Returns (results, summary).  progress(msg)
        is called every `progress_every` ticks."""
        order = sorted(range(len(requests)), key=lambda i: arrivals[i])
        queue = []             # arrived, waiting for admission (FIFO)
        resident = {}          # slot -> request index
        results = [None] * len(requests)
        admitted_at = {}
        nxt = 0
        t0 = self.clock()
        peak_bytes = 0
        resident_bytes = 0
        ticks = 0
        admit_order = []
        while nxt < len(order) or queue or resident:
            now = self.clock() - t0
            if max_wall is not None and now > max_wall:
                raise TimeoutError("serving loop exceeded %.1f s" % max_wall)
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                queue.append(order[nxt])
                nxt += 1
            # admit from the head while it fits
            while queue:
                i = queue[0]
                need = self.footprint(requests[i])
                if self.heap_bytes is not None and need > self.heap_bytes:
                    results[i] = dict(request=i, rejected=True, reason="footprint %d > heap %d" % (need, self.heap_bytes))
                    queue.pop(0)
                    continue
                slot = self.engine.admit(requests[i])
                if slot is None:
                    break
                queue.pop(0)
                resident[slot] = i
                admitted_at[i] = self.clock() - t0
                admit_order.append(i)
                resident_bytes += need
                peak_bytes = max(peak_bytes, resident_bytes)
            if resident:
                self.engine.run(1)
                ticks += 1
                if progress is not None and ticks % progress_every == 0:
                    n_done = sum(1 for r in results if r is not None)
                    progress("tick %d t=%.1fs resident=%d queued=%d done=%d" % (ticks, self.clock() - t0, len(resident),
                                                                                len(queue), n_done))
                done, _ = self.engine.poll()
                for slot in done:
                    i = resident.pop(slot)
                    out = self.engine.fetch(slot)
                    self.engine.release(slot)
                    resident_bytes -= self.footprint(requests[i])
                    t_done = self.clock() - t0
                    c = requests[i]
                    cells = int(c["nx"]) * int(c["ny"]) * int(c["nz"])
                    r = dict(request=i, rejected=False, arrival=arrivals[i], admitted=admitted_at[i], done=t_done,
                             latency=t_done - arrivals[i], k_f=out["k_f"], status=out["status"], cells=cells,
                             cell_iters=cells * (1 + out["k_f"]))
                    if keep_fields:
                        r.update(alpha=out["alpha"], p=out["p"], U=out["U"])
                    results[i] = r
            elif nxt < len(order):
                wait = arrivals[order[nxt]] - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 0.05))
        wall = self.clock() - t0
        served = [r for r in results if r and not r["rejected"]]
        lat = [r["latency"] for r in served]
        summary = dict(requests=len(requests), served=len(served), rejected=len(requests) - len(served),
                       wall_s=wall, ticks=ticks, peak_resident_bytes=peak_bytes,
                       p50_latency_s=nearest_rank(lat, 50), p99_latency_s=nearest_rank(lat, 99),
                       mcell_iter_per_s=sum(r["cell_iters"] for r in served) / wall / 1e6 if wall > 0 else 0.0,
                       admit_order=admit_order)
        return results, summary
