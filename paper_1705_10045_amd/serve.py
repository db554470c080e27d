"""Continuous-batching serving loop over the device pool (lbm_pool_* in the C ABI).

Requests (independent D3Q19 thermal two-phase simulations of uneven lattice sizes) arrive over
time.  The loop admits every arrived request that fits a free slot and the remaining HBM
budget (first fit in arrival order), advances all admitted requests together with one pool
replay (one batched launch per step, replayed from a HIP graph), collects the finished ones
and frees their slots for the requests still waiting.  With the device pool the replay is left
in flight while the loop collects and admits, so host work and uploads overlap the device's
steps.  Time-to-result of a request is the time its result fields reach the caller minus its
arrival time.

The scheduler is written against a small executor interface (submit / run / poll / collect /
stats) so that its bookkeeping can be exercised without a device; `PoolExecutor` is the real
one, backed by the HIP library.
"""
import collections
import math
import time

import numpy as np

from . import inputs


def poisson_arrivals(count, rate, seed=inputs.SEED):
    """Arrival times (seconds from 0) of a Poisson process of the given rate (requests/s),
    from counter-based uniforms (exponential gaps by inversion)."""
    if rate <= 0 or math.isinf(rate):
        return np.zeros(count)
    u = inputs.uniform(seed + 77, count)
    gaps = -np.log(1.0 - u) / rate
    return np.cumsum(gaps) - gaps[0]


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


# bytes of the two FP32 D3Q19 population buffers of an L^3 request, without plane padding:
# a lower bound of what the pool's arena must hold for it
def request_bytes_lower_bound(edge):
    return 2 * 2 * 19 * 4 * edge ** 3


class PoolExecutor:
    """Executor backed by the device pool.  A request that cannot fit (no free slot, or fewer
    free arena bytes than its buffers need) is declined without building its fields; a
    request's initial fields are built once and kept until it is admitted.  `payload`, if
    given, maps a request id to fields that arrived with the request (built by the client)."""

    def __init__(self, pool, physics=None, payload=None):
        self.pool = pool
        self.physics = physics or inputs.physics()
        self._fields = dict(payload) if payload else {}

    def submit(self, req):
        st = self.pool.stats()
        if st["free_slots"] < 1 or (st["budget"] - st["bytes_in_use"] <
                                    request_bytes_lower_bound(req["edge"])):
            return None
        f = self._fields.get(req["id"])
        if f is None:
            f = self._fields[req["id"]] = inputs.request_fields(req, self.physics)
        ticket = self.pool.submit(f["params"], f["rho0"], f["u0"], f["T0"], req["steps"])
        if ticket is not None:
            del self._fields[req["id"]]
        return ticket

    def run(self):
        # the replay stays in flight while the loop collects, admits and uploads (on the pool's
        # second stream); the next call waits for it
        self.pool.run_async()

    def poll(self, ticket):
        return self.pool.poll(ticket)

    def collect(self, ticket):
        return self.pool.collect(ticket)

    def stats(self):
        return self.pool.stats()


def serve(requests, arrivals, executor, clock=time.perf_counter, sleep=time.sleep,
          keep_results=False, progress=None):
    """Run the continuous-batching loop.  Returns a report dict with per-request latencies,
    p50/p99 time-to-result, aggregate node updates per second and the peak number of requests
    in flight.  `requests[i]` arrives at `arrivals[i]` seconds after the start.  `progress`,
    if given, is called with the number of completed requests after each completion."""
    order = sorted(range(len(requests)), key=lambda i: (arrivals[i], i))
    pending = collections.deque(order)
    waiting = []                         # arrived, not yet admitted (arrival order)
    inflight = {}                        # ticket -> request index
    latency = {}
    status = {}
    results = {}
    node_updates = 0
    peak = 0
    replays = 0
    t0 = clock()
    while pending or waiting or inflight:
        now = clock() - t0
        while pending and arrivals[pending[0]] <= now:
            waiting.append(pending.popleft())
        still = []
        for i in waiting:                # first fit in arrival order
            ticket = executor.submit(requests[i])
            if ticket is None:
                still.append(i)
            else:
                inflight[ticket] = i
        waiting = still
        peak = max(peak, len(inflight))
        if not inflight:
            if pending:
                sleep(max(0.0, arrivals[pending[0]] - (clock() - t0)))
            elif waiting:
                raise RuntimeError("request %d can never be admitted (larger than the pool)"
                                   % requests[waiting[0]]["id"])
            continue
        executor.run()
        replays += 1
        for ticket in list(inflight):
            done, st = executor.poll(ticket)
            if not done:
                continue
            i = inflight.pop(ticket)
            fields, st = executor.collect(ticket)
            # time-to-result includes delivering the result fields to the caller
            latency[i] = clock() - t0 - arrivals[i]
            status[i] = st
            if keep_results:
                results[i] = fields
            if st == 0:
                r = requests[i]
                node_updates += r["edge"] ** 3 * r["steps"]
            if progress:
                progress(len(latency))
    wall = clock() - t0
    lat = [latency[i] for i in range(len(requests)) if status.get(i) == 0]
    report = {
        "requests": len(requests), "completed": len(lat),
        "failed": sum(1 for s in status.values() if s != 0),
        "wall_s": wall, "replays": replays, "peak_in_flight": peak,
        "node_updates": node_updates,
        "aggregate_mlups": node_updates / wall / 1e6 if wall > 0 else float("nan"),
        "p50_s": percentile(lat, 50) if lat else None,
        "p99_s": percentile(lat, 99) if lat else None,
        "latency_s": [latency.get(i) for i in range(len(requests))],
        "status": [status.get(i) for i in range(len(requests))],
    }
    if keep_results:
        report["results"] = results
    return report


def one_at_a_time(requests, physics=None, clock=time.perf_counter, payload=None, progress=None):
    """The same requests solved one after another with a single simulation each (lbm_init,
    lbm_step, lbm_moments, lbm_free): aggregate node updates per second.  `payload` as for
    PoolExecutor; `progress` as for serve.  A request that leaves the EOS domain counts as
    failed (its time counts, its node updates do not), as in the pool."""
    from . import lbm
    physics = physics or inputs.physics()
    t0 = clock()
    total = 0
    failed = []
    for n_done, r in enumerate(requests, 1):
        f = payload[r["id"]] if payload else inputs.request_fields(r, physics)
        with lbm.Sim(19, f["params"], f["rho0"], f["u0"], f["T0"], storage_bytes=4) as s:
            try:
                s.step(r["steps"])
                s.moments()
                total += r["edge"] ** 3 * r["steps"]
            except lbm.LbmError as e:
                if e.status != lbm.LBM_EUNSTABLE:
                    raise
                failed.append(r["id"])
        if progress:
            progress(n_done)
    wall = clock() - t0
    return {"wall_s": wall, "node_updates": total, "aggregate_mlups": total / wall / 1e6,
            "failed_ids": failed}
