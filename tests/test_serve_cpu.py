"""The continuous-batching scheduler on the CPU, with a fake executor and a
virtual clock: per-run FIFO order, continuous batching (requests that arrive
while a micro-batch is on the device join the next one), admission waits and
evictions under a small footprint budget, and latency accounting."""
import numpy as np

from paper_2606_29692_amd.serve import Executor, Request, Server, latency_summary, poisson_trace


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    """Each launch takes `dt` virtual seconds; results encode (run, step)."""

    def __init__(self, keys: dict, slots: int, dt: float, clock: Clock, fp: int = 100):
        self.keys, self.slots, self.dt, self.clock, self.fp = keys, slots, dt, clock, fp
        self.finish = {}
        self.launches = []
        self.resident = set()
        self.admits = 0
        self.steps = {r: 0 for r in keys}

    def groups(self):
        return {k: self.slots for k in set(self.keys.values())}

    def run_key(self, run):
        return self.keys[run]

    def footprint(self, run):
        return self.fp

    def fixed_bytes(self):
        return 0

    def admit(self, run):
        assert run not in self.resident
        self.resident.add(run)
        self.admits += 1

    def evict(self, run):
        self.resident.remove(run)

    def launch(self, key, batch):
        assert key not in self.finish or self.finish[key] <= self.clock.t
        for run, slot, th in batch:
            assert run in self.resident
            assert self.keys[run] == key
        assert len({s for _, s, _ in batch}) == len(batch)
        self.launches.append((self.clock.t, key, list(batch)))
        self.finish[key] = self.clock.t + self.dt

    def done(self, key):
        return self.finish.get(key, 0.0) <= self.clock.t

    def results(self, key, batch):
        out = []
        for run, slot in batch:
            out.append((float(run), self.steps[run], 0.0))
            self.steps[run] += 1
        return out


def drive(server, clock, reqs, dt_tick=1e-4, t_end=100.0):
    pending = sorted(reqs, key=lambda q: q.t_arrival)
    i = 0
    while len(server.completed) < len(reqs) and clock.t < t_end:
        while i < len(pending) and pending[i].t_arrival <= clock.t:
            server.submit(pending[i])
            i += 1
        server.poll()
        server.schedule()
        clock.t += dt_tick
    return pending


def test_fifo_per_run_and_continuous_batching():
    clock = Clock()
    keys = {r: (8 + 2 * (r % 2),) for r in range(6)}
    ex = FakeExecutor(keys, slots=4, dt=1e-3, clock=clock)
    server = Server(ex, {r: np.arange(50) * 0.01 for r in keys}, budget_bytes=10**9, clock=clock)
    reqs = poisson_trace(200, rate=3000.0, n_runs=6, seed=1)
    drive(server, clock, reqs)
    assert len(server.completed) == 200
    # per-run FIFO: a run's k-th completed request is its k-th arrival
    for r in keys:
        mine = [q for q in reqs if q.run == r]
        assert [q.selected for q in mine] == list(range(len(mine)))
        assert all(a.t_done <= b.t_start for a, b in zip(mine, mine[1:]))
    # continuous batching: micro-batches hold several runs, and requests that
    # arrived while a launch was running start right when it completes
    assert max(len(b) for _, _, b in ex.launches) > 1
    for q in reqs:
        assert q.t_start >= q.t_arrival and q.t_done >= q.t_start + 1e-3 - 1e-9
    # the angle handed to each launch is the run's next one
    for t, key, batch in ex.launches:
        for run, slot, th in batch:
            assert 0.0 <= th < 0.5


def test_admission_waits_and_evictions_under_small_budget():
    clock = Clock()
    keys = {r: (10,) for r in range(8)}
    ex = FakeExecutor(keys, slots=8, dt=5e-4, clock=clock, fp=100)
    server = Server(ex, {r: np.zeros(10) for r in keys}, budget_bytes=250, clock=clock)
    reqs = [Request(i, i % 8, 1e-4 * i) for i in range(64)]
    drive(server, clock, reqs)
    assert len(server.completed) == 64
    assert server.evictions > 0 and server.admission_waits > 0
    assert ex.admits > 8                          # evicted runs came back
    assert server.used <= 250
    for r in keys:
        mine = [q for q in reqs if q.run == r]
        assert [q.selected for q in mine] == list(range(len(mine)))
    assert any(q.cold for q in reqs)


def test_latency_summary():
    reqs = [Request(i, 0, 0.001 * i) for i in range(100)]
    for q in reqs:
        q.t_start = q.t_arrival
        q.t_done = q.t_arrival + 0.002
    s = latency_summary(reqs)
    assert abs(s["p50_ms"] - 2.0) < 1e-9 and abs(s["p99_ms"] - 2.0) < 1e-9
    assert s["n"] == 100
