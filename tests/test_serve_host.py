"""Host-side scheduling of the serving loop, with a stand-in engine and a
simulated clock (no GPU): arrivals are submitted once their time has passed,
capacity limits how many requests iterate together, every request finishes,
and latency counts the wait for a slot."""
import numpy as np

from paper_2603_01064_amd.serve import serve_requests, serve_serially


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeEngine:
    """Capacity-limited engine: request i needs need[i] steps; a step costs dt."""

    def __init__(self, capacity, need, clock, dt):
        self.capacity, self.need, self.clock, self.dt = capacity, need, clock, dt
        self.queue, self.active = [], {}
        self.max_active = 0

    def serve_submit(self, b, x, alpha, ws, rid):
        self.queue.append(rid)

    def serve_pending(self):
        return len(self.queue), len(self.active)

    def serve_step(self, **kw):
        while self.queue and len(self.active) < self.capacity:
            self.active[self.queue.pop(0)] = 0
        self.max_active = max(self.max_active, len(self.active))
        done = []
        for rid in list(self.active):
            if self.active[rid] >= self.need[rid]:
                done.append(type("R", (), {"id": rid, "cycles": self.active[rid], "status": 0})())
                del self.active[rid]
        for rid in self.active:
            self.active[rid] += 1
        self.clock.t += self.dt
        return done


def test_all_requests_finish_with_capacity_respected():
    rng = np.random.default_rng(0)
    n = 40
    need = rng.integers(3, 12, size=n)
    arrivals = np.cumsum(rng.exponential(0.002, size=n))
    clk = FakeClock()
    eng = FakeEngine(4, need, clk, 0.001)
    rep = serve_requests(eng, [None] * n, [None] * n, np.ones(n), np.zeros(n, dtype=int), arrivals, clock=clk,
                         sleep=clk.sleep)
    assert (rep.status == 0).all()
    assert np.array_equal(rep.cycles, need)
    assert eng.max_active <= 4
    # a request cannot finish before it has iterated need[i] times after arriving
    assert (rep.latency_ms >= 1e3 * need * 0.001 - 1e-9).all()
    s = rep.summary()
    assert s["requests"] == n and s["converged"] == n and s["p99_ms"] >= s["p50_ms"]


def test_idle_engine_waits_for_the_next_arrival():
    clk = FakeClock()
    eng = FakeEngine(8, [2, 2], clk, 0.001)
    rep = serve_requests(eng, [None] * 2, [None] * 2, np.ones(2), np.zeros(2, dtype=int), np.array([0.0, 5.0]),
                         clock=clk, sleep=clk.sleep)
    # the second request arrives long after the first finished: its latency is its own 3 steps
    assert abs(rep.latency_ms[1] - 3.0) < 1e-6
    assert rep.steps == 6


def test_serial_baseline_queues_in_arrival_order():
    clk = FakeClock()

    def solve_one(i):
        clk.t += 0.010
        return 5, 0

    rep = serve_serially(solve_one, np.array([0.0, 0.001, 0.002]), clock=clk, sleep=clk.sleep)
    assert np.allclose(rep.latency_ms, [10.0, 19.0, 28.0])
