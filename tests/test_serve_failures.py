"""Failure handling of the continuous-batching server, on the CPU (fake
executor, virtual clock): a run whose admission fails (an operator with a
mask bit outside the register, which the library refuses with VQE_EINVAL; an
injected allocation failure raised through the binding's hook as VQE_ENOMEM),
a request with a non-finite angle (VQE_EINVAL on the host, before any launch),
and a launch that raises.  In every case the failed requests complete with
their error and status, the other runs keep serving in order, and the
latency figures leave the failures out."""
import numpy as np
import pytest

from paper_2606_29692_amd import binding as B
from paper_2606_29692_amd.serve import Request, Server, latency_summary

from test_serve_cpu import Clock, FakeExecutor, drive


class PackExecutor(FakeExecutor):
    """Fake executor whose admission checks each run's Pauli pack the way the
    CSR builder does (every mask bit below the register size, else
    VQE_EINVAL) and passes through the binding's allocation hook."""

    def __init__(self, keys, packs, *a, fail_launch_at=None, **kw):
        super().__init__(keys, *a, **kw)
        self.packs = packs
        self.fail_launch_at = fail_launch_at
        self.n_launch = 0
        self.released = []

    def admit(self, run):
        n_q, x, z = self.packs[run]
        if np.any((np.asarray(x, dtype=np.uint64) | np.asarray(z, dtype=np.uint64)) >> np.uint64(n_q)):
            raise B.VqeError(B.VQE_EINVAL, f"csr_build_from_pauli: mask bit >= n_qubits")
        B.check_fault("alloc")
        super().admit(run)

    def launch(self, key, batch):
        self.n_launch += 1
        if self.fail_launch_at is not None and self.n_launch == self.fail_launch_at:
            raise B.VqeError(B.VQE_EHIP, "vqe_batch_step: injected launch failure")
        super().launch(key, batch)

    def release(self, key, slot):
        self.released.append((key, slot))


def packs_for(keys, bad=()):
    out = {}
    for r, key in keys.items():
        n_q = key[0]
        x = np.array([1, 3], dtype=np.uint64)
        z = np.array([0, 1 << n_q if r in bad else 2], dtype=np.uint64)
        out[r] = (n_q, x, z)
    return out


def by_run(reqs, r):
    return [q for q in reqs if q.run == r]


def test_bad_operator_fails_its_run_only():
    clock = Clock()
    keys = {r: (8,) for r in range(4)}
    ex = PackExecutor(keys, packs_for(keys, bad={2}), slots=4, dt=1e-3, clock=clock)
    server = Server(ex, {r: np.full(20, 0.05) for r in keys}, budget_bytes=10**9, clock=clock)
    reqs = [Request(i, i % 4, 1e-4 * i) for i in range(40)]
    drive(server, clock, reqs)
    assert len(server.completed) == 40
    bad = by_run(reqs, 2)
    assert all(q.failed and q.status == B.VQE_EINVAL and "mask bit" in q.error for q in bad)
    for r in (0, 1, 3):
        mine = by_run(reqs, r)
        assert not any(q.failed for q in mine)
        assert [q.selected for q in mine] == list(range(len(mine)))
    s = latency_summary(reqs)
    assert s["failed"] == len(bad) and s["n"] == 40 - len(bad)


def test_injected_allocation_failure_through_the_binding():
    clock = Clock()
    keys = {r: (10,) for r in range(3)}
    ex = PackExecutor(keys, packs_for(keys), slots=4, dt=1e-3, clock=clock)
    server = Server(ex, {r: np.full(20, 0.05) for r in keys}, budget_bytes=10**9, clock=clock)
    B.inject_fault("alloc", 1)
    try:
        reqs = [Request(i, i % 3, 1e-4 * i) for i in range(30)]
        drive(server, clock, reqs)
    finally:
        B.inject_fault("alloc", 0)
    failed_runs = {q.run for q in reqs if q.failed}
    assert len(failed_runs) == 1                    # the first admission hit the fault
    (fr,) = failed_runs
    assert all(q.status == B.VQE_ENOMEM for q in by_run(reqs, fr))
    for r in set(keys) - failed_runs:
        mine = by_run(reqs, r)
        assert not any(q.failed for q in mine)
        assert [q.selected for q in mine] == list(range(len(mine)))


def test_non_finite_angle_is_refused_before_launch():
    clock = Clock()
    keys = {r: (8,) for r in range(2)}
    ex = PackExecutor(keys, packs_for(keys), slots=2, dt=1e-3, clock=clock)
    server = Server(ex, {r: np.full(20, 0.05) for r in keys}, budget_bytes=10**9, clock=clock)
    reqs = [Request(i, i % 2, 1e-4 * i) for i in range(12)]
    reqs[4].theta = float("nan")
    reqs[7].theta = float("inf")
    drive(server, clock, reqs)
    assert len(server.completed) == 12
    assert reqs[4].failed and reqs[4].status == B.VQE_EINVAL
    assert reqs[7].failed and reqs[7].status == B.VQE_EINVAL
    launched = [th for _, _, b in ex.launches for _, _, th in b]
    assert all(np.isfinite(launched))
    # a refused request does not advance its run: the next one takes the next step
    for r in keys:
        ok = [q for q in by_run(reqs, r) if not q.failed]
        assert [q.selected for q in ok] == list(range(len(ok)))


def test_launch_failure_fails_that_micro_batch_and_serving_continues():
    clock = Clock()
    keys = {r: (12,) for r in range(4)}
    ex = PackExecutor(keys, packs_for(keys), slots=4, dt=1e-3, clock=clock, fail_launch_at=2)
    server = Server(ex, {r: np.full(30, 0.05) for r in keys}, budget_bytes=10**9, clock=clock)
    reqs = [Request(i, i % 4, 2e-4 * i) for i in range(40)]
    drive(server, clock, reqs)
    assert len(server.completed) == 40
    failed = [q for q in reqs if q.failed]
    assert failed and all(q.status == B.VQE_EHIP and "launch failed" in q.error for q in failed)
    assert len(ex.released) == len(failed)         # their slots were unbound
    assert not any(server.runs[r].busy for r in keys)
    # later requests of the same runs were served
    for q in failed:
        assert any(not p.failed and p.t_arrival > q.t_arrival for p in by_run(reqs, q.run))


def test_budget_too_small_for_a_run_fails_it_instead_of_stopping():
    clock = Clock()
    keys = {0: (8,), 1: (8,)}
    ex = PackExecutor(keys, packs_for(keys), slots=2, dt=1e-3, clock=clock, fp=500)
    server = Server(ex, {r: np.full(5, 0.05) for r in keys}, budget_bytes=100, clock=clock)
    reqs = [Request(i, i % 2, 1e-4 * i) for i in range(6)]
    drive(server, clock, reqs)
    assert all(q.failed and q.status == -3 for q in reqs)


@pytest.mark.parametrize("spec,n", [("alloc:2", 2), ("alloc", 1)])
def test_fault_from_environment(monkeypatch, spec, n):
    monkeypatch.setenv("ADAPTVQE_FAULT", spec)
    B._arm_from_env()
    hits = 0
    for _ in range(n + 2):
        try:
            B.check_fault("alloc")
        except B.VqeError as e:
            assert e.status == B.VQE_ENOMEM
            hits += 1
    assert hits == n
