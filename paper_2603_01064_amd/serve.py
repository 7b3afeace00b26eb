"""Request-driven serving loop over the library's continuous-batching engine.

Requests arrive at given times (seconds from the start); each is submitted to
the handle as soon as the host sees that its arrival time has passed, and the
loop steps the engine (one outer iteration for every request in flight)
while any request is queued or active.  A request's latency is the wall time
from its arrival to the end of the step that retired it, so it includes the
time it waited for a free batch slot.

Only the arrival clock lives here: admission, the iteration and retirement
run in the HIP library (``nmg_serve_step`` for one handle, ``nmg_pool_step``
for a pool of handles of different grid sizes under one memory budget).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np


@dataclass
class ServeReport:
    latency_ms: np.ndarray   # per request, in submission order
    cycles: np.ndarray
    status: np.ndarray
    wall_s: float            # first arrival to last completion
    steps: int

    def summary(self) -> dict:
        ok = self.status == 0
        lat = self.latency_ms[ok] if ok.any() else np.array([np.nan])
        return {"requests": int(self.latency_ms.size), "converged": int(ok.sum()),
                "solves_per_s": round(float(self.latency_ms.size / self.wall_s), 2) if self.wall_s > 0 else None,
                "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_cycles": round(float(self.cycles.mean()), 2), "engine_steps": int(self.steps),
                "status_counts": {str(int(v)): int((self.status == v).sum()) for v in np.unique(self.status)}}


def serve_requests(handle, b, x, alpha, weight_set, arrivals, *, rtol=1e-6, max_cycles=200, nu1=1, nu2=1,
                   use_fprime=False, precision="mixed", clock=time.perf_counter, sleep=time.sleep) -> ServeReport:
    """Serves ``len(arrivals)`` requests: request ``i`` solves ``b[i]`` into
    ``x[i]`` with ``alpha[i]`` and smoother set ``weight_set[i]`` and becomes
    visible at ``arrivals[i]`` seconds (non-decreasing) after the start."""
    count = len(arrivals)
    lat = np.full(count, np.nan)
    cyc = np.zeros(count, dtype=np.int64)
    status = np.full(count, -1, dtype=np.int64)
    finished = 0
    nxt = 0
    steps = 0
    t0 = clock()
    while finished < count:
        now = clock() - t0
        while nxt < count and arrivals[nxt] <= now:
            handle.serve_submit(b[nxt], x[nxt], float(alpha[nxt]), int(weight_set[nxt]), rid=nxt)
            nxt += 1
        queued, active = handle.serve_pending()
        if queued + active == 0:
            sleep(max(0.0, float(arrivals[nxt]) - (clock() - t0)))
            continue
        done = handle.serve_step(rtol=rtol, max_cycles=max_cycles, nu1=nu1, nu2=nu2, use_fprime=use_fprime,
                                 precision=precision)
        steps += 1
        t_done = clock() - t0
        for r in done:
            i = int(r.id)
            lat[i] = 1e3 * (t_done - float(arrivals[i]))
            cyc[i] = int(r.cycles)
            status[i] = int(r.status)
            finished += 1
    wall = (clock() - t0) - float(arrivals[0]) if count else 0.0
    return ServeReport(latency_ms=lat, cycles=cyc, status=status, wall_s=wall, steps=steps)


def serve_serially(solve_one, arrivals, clock=time.perf_counter, sleep=time.sleep) -> ServeReport:
    """The one-request-at-a-time baseline on the same arrival trace:
    ``solve_one(i) -> (cycles, status)`` solves request ``i`` to completion;
    requests wait in arrival order while an earlier one is being solved."""
    count = len(arrivals)
    lat = np.full(count, np.nan)
    cyc = np.zeros(count, dtype=np.int64)
    status = np.full(count, -1, dtype=np.int64)
    t0 = clock()
    for i in range(count):
        wait = float(arrivals[i]) - (clock() - t0)
        if wait > 0:
            sleep(wait)
        c, st = solve_one(i)
        lat[i] = 1e3 * ((clock() - t0) - float(arrivals[i]))
        cyc[i] = c
        status[i] = st
    wall = (clock() - t0) - float(arrivals[0]) if count else 0.0
    return ServeReport(latency_ms=lat, cycles=cyc, status=status, wall_s=wall, steps=count)


def serve_pool_requests(pool, member, b, x, alpha, weight_set, arrivals, *, rtol=1e-6, max_cycles=200, nu1=1,
                        nu2=1, use_fprime=False, precision="mixed", clock=time.perf_counter,
                        sleep=time.sleep) -> ServeReport:
    """As :func:`serve_requests` over a :class:`nmg.Pool`: request ``i`` goes
    to pool member ``member[i]`` (its grid size) with ``b[i]``/``x[i]`` of
    that member's shape.  Latency counts from the arrival time."""
    count = len(arrivals)
    lat = np.full(count, np.nan)
    cyc = np.zeros(count, dtype=np.int64)
    status = np.full(count, -1, dtype=np.int64)
    finished = nxt = steps = 0
    t0 = clock()
    while finished < count:
        now = clock() - t0
        while nxt < count and arrivals[nxt] <= now:
            pool.submit(int(member[nxt]), b[nxt], x[nxt], float(alpha[nxt]), int(weight_set[nxt]), rid=nxt)
            nxt += 1
        queued, active, _ = pool.pending()
        if queued + active == 0:
            sleep(max(0.0, float(arrivals[nxt]) - (clock() - t0)))
            continue
        done = pool.step(rtol=rtol, max_cycles=max_cycles, nu1=nu1, nu2=nu2, use_fprime=use_fprime,
                         precision=precision)
        steps += 1
        t_done = clock() - t0
        for _, r in done:
            i = int(r.id)
            lat[i] = 1e3 * (t_done - float(arrivals[i]))
            cyc[i] = int(r.cycles)
            status[i] = int(r.status)
            finished += 1
    wall = (clock() - t0) - float(arrivals[0]) if count else 0.0
    return ServeReport(latency_ms=lat, cycles=cyc, status=status, wall_s=wall, steps=steps)
