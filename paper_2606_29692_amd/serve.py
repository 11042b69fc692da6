"""Continuous-batching request loop for adaptive-VQE runs.

A *run* is one adaptive simulation (its Hamiltonian, pool and state vector);
a *request* asks for the run's next adaptive step (energy, pool-gradient
screen, selection, Taylor-5 update, renormalisation).  A run's requests are
served in arrival order, one at a time.

Device side: one *slot group* per register size, each a batch plan with a
fixed number of slots, its own HIP stream and its captured graphs.  Runs are
bound to free slots with ``vqe_batch_rebind`` and switched on through the
plan's activity flags, so a micro-batch of any composition replays the same
graphs.  Groups run on separate streams: their work overlaps on the device.

Host side (``Server``): requests arrive, runs are admitted to the device when
their HBM footprint fits the budget (idle runs are evicted, least recently
used first, their state copied to the host and restored on return), each idle
slot group launches a micro-batch of the oldest ready requests as soon as its
previous micro-batch completes, and completions are polled without blocking.
Latencies are host-observed (arrival to completion seen by the loop).

Failures: a request whose angle is not finite is failed on the host before
any launch (status EINVAL, as the library would return); a run whose
admission raises (its operator cannot be built: bad masks, out of memory) is
marked failed with all its queued requests, and later requests for it fail at
once; a launch or result read-back that raises fails the requests of that
micro-batch, frees their slots and leaves every other run serving.  Failed
requests complete with ``error`` set and are kept out of the latency figures.

The scheduling logic is written against the ``Executor`` interface so it can
be exercised without a GPU; ``DeviceExecutor`` is the HIP implementation.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    run: int
    t_arrival: float
    t_start: float | None = None
    t_done: float | None = None
    energy: float | None = None
    selected: int | None = None
    gmax: float | None = None
    cold: bool = False              # the run had to be (re)built on the device first
    theta: float | None = None      # angle of this step (default: the run's next angle)
    error: str | None = None        # set when the request failed
    status: int = 0                 # library status of a failure (negative), else 0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def failed(self) -> bool:
        return self.error is not None


@dataclass
class RunState:
    run: int
    key: tuple                      # slot-group key (register size)
    footprint: int                  # device bytes while resident
    thetas: np.ndarray              # angle of each successive step
    step: int = 0
    resident: bool = False
    busy: bool = False
    queue: collections.deque = field(default_factory=collections.deque)
    last_used: float = 0.0
    failed: str | None = None       # admission failed: the run serves no more requests
    failed_status: int = 0


class Executor:
    """What the scheduler needs from the device."""

    def groups(self) -> dict:                       # key -> number of slots
        raise NotImplementedError

    def run_key(self, run: int) -> tuple:
        raise NotImplementedError

    def footprint(self, run: int) -> int:
        raise NotImplementedError

    def fixed_bytes(self) -> int:
        raise NotImplementedError

    def admit(self, run: int):                      # make the run resident
        raise NotImplementedError

    def evict(self, run: int):                      # release its device memory
        raise NotImplementedError

    def launch(self, key: tuple, batch: list):      # batch: [(run, slot, theta)]
        raise NotImplementedError

    def done(self, key: tuple) -> bool:             # previous launch of the group finished
        raise NotImplementedError

    def results(self, key: tuple, batch: list) -> list:   # [(energy, k, gmax)]
        raise NotImplementedError

    def release(self, key: tuple, slot: int):       # a failed slot: unbind it (optional)
        pass


class Server:
    """Continuous batching over slot groups with admission by HBM footprint."""

    def __init__(self, executor: Executor, thetas: dict, budget_bytes: int,
                 clock=time.perf_counter):
        self.ex = executor
        self.clock = clock
        self.budget = int(budget_bytes)
        self.used = executor.fixed_bytes()
        self.runs = {r: RunState(r, executor.run_key(r), executor.footprint(r), np.asarray(th))
                     for r, th in thetas.items()}
        self.slots = {k: [None] * n for k, n in executor.groups().items()}   # slot -> run
        self.by_key = collections.defaultdict(list)
        for r in self.runs.values():
            self.by_key[r.key].append(r)
        self.inflight: dict = {}            # key -> list of (req, slot)
        self.completed: list = []
        self.failed: list = []
        self.admission_waits = 0
        self.evictions = 0

    @property
    def failed_count(self) -> int:
        return len(self.failed)

    # ------------------------------------------------------------------ failures
    def _fail(self, req: Request, msg: str, status: int):
        now = self.clock()
        if req.t_start is None:
            req.t_start = now
        req.t_done = now
        req.error, req.status = msg, int(status)
        self.completed.append(req)
        self.failed.append(req)

    def _fail_run(self, r: RunState, msg: str, status: int):
        """Mark a run failed and fail every request queued for it."""
        r.failed, r.failed_status = msg, int(status)
        r.busy = False
        while r.queue:
            self._fail(r.queue.popleft(), msg, status)

    def _release(self, key: tuple, slot: int):
        slots = self.slots[key]
        slots[slot] = None
        try:
            self.ex.release(key, slot)
        except Exception:       # noqa: BLE001 (a release failure must not stop serving)
            pass

    # ------------------------------------------------------------------ requests
    def submit(self, req: Request):
        r = self.runs[req.run]
        if r.failed is not None:
            self._fail(req, r.failed, r.failed_status)
            return
        r.queue.append(req)

    def pending(self) -> int:
        return sum(len(r.queue) for r in self.runs.values()) + sum(
            len(v) for v in self.inflight.values())

    # ------------------------------------------------------------------ memory
    def _make_room(self, need: int) -> bool:
        if self.used + need <= self.budget:
            return True
        idle = [r for r in self.runs.values() if r.resident and not r.busy and not r.queue]
        idle.sort(key=lambda r: r.last_used)
        for r in idle:
            self.ex.evict(r.run)
            r.resident = False
            self.used -= r.footprint
            self.evictions += 1
            slots = self.slots[r.key]
            for i, occ in enumerate(slots):
                if occ == r.run:
                    slots[i] = None
            if self.used + need <= self.budget:
                return True
        return False

    def _admit(self, r: RunState) -> bool:
        if r.resident:
            return True
        if r.footprint > self.budget - self.ex.fixed_bytes():
            self._fail_run(r, f"run {r.run} needs {r.footprint} bytes: more than the budget "
                              f"leaves after the fixed {self.ex.fixed_bytes()} bytes",
                           STATUS_ENOMEM)
            return False
        if not self._make_room(r.footprint):
            self.admission_waits += 1
            return False
        try:
            self.ex.admit(r.run)
        except (RuntimeError, ValueError, MemoryError) as e:
            self._fail_run(r, f"admission of run {r.run} failed: {e}", _status_of(e))
            return False
        r.resident = True
        r.footprint = self.ex.footprint(r.run)      # the built size replaces the estimate
        self.used += r.footprint
        return True

    def prewarm(self) -> int:
        """Admit runs (in run order) while the budget allows; returns how many
        are resident.  Serving then starts warm: CSRs and states on the device."""
        n = 0
        for r in sorted(self.runs.values(), key=lambda r: r.run):
            if r.resident:
                n += 1
                continue
            if self.used + r.footprint > self.budget:
                continue
            try:
                self.ex.admit(r.run)
            except (RuntimeError, ValueError, MemoryError) as e:
                self._fail_run(r, f"admission of run {r.run} failed: {e}", _status_of(e))
                continue
            r.resident = True
            r.footprint = self.ex.footprint(r.run)
            self.used += r.footprint
            n += 1
        return n

    # ------------------------------------------------------------------ scheduling
    def poll(self):
        now = self.clock()
        for key in list(self.inflight):
            if self.ex.done(key):
                batch = self.inflight.pop(key)
                try:
                    res = self.ex.results(key, [(req.run, slot) for req, slot in batch])
                except (RuntimeError, ValueError) as e:
                    self._fail_batch(key, batch, f"result read-back failed: {e}", _status_of(e))
                    continue
                now = self.clock()
                for (req, slot), (e, k, gm) in zip(batch, res):
                    req.t_done = now
                    req.energy, req.selected, req.gmax = e, k, gm
                    r = self.runs[req.run]
                    r.busy = False
                    r.step += 1
                    r.last_used = now
                    self.completed.append(req)

    def _fail_batch(self, key: tuple, batch: list, msg: str, status: int):
        for req, slot in batch:
            r = self.runs[req.run]
            r.busy = False
            self._release(key, slot)
            self._fail(req, msg, status)

    def schedule(self):
        for key, slots in self.slots.items():
            if key in self.inflight:
                continue
            ready = [r for r in self.by_key[key] if r.queue and not r.busy and r.failed is None]
            if not ready:
                continue
            ready.sort(key=lambda r: r.queue[0].t_arrival)
            batch = []
            taken = set()
            for r in ready:
                if len(batch) == len(slots):
                    break
                head = r.queue[0]
                th = head.theta if head.theta is not None else float(r.thetas[r.step % len(r.thetas)])
                if not np.isfinite(th):
                    # the library refuses a non-finite angle (VQE_EINVAL); fail it here
                    self._fail(r.queue.popleft(), f"request {head.rid}: non-finite angle {th}",
                               STATUS_EINVAL)
                    continue
                cold = not r.resident
                if not self._admit(r):
                    continue
                slot = next((i for i, occ in enumerate(slots) if occ == r.run), None)
                if slot is None:
                    slot = next((i for i, occ in enumerate(slots)
                                 if i not in taken and (occ is None or not self._in_use(occ))), None)
                if slot is None:
                    continue
                slots[slot] = r.run
                taken.add(slot)
                req = r.queue.popleft()
                req.t_start = self.clock()
                req.cold = cold
                r.busy = True
                batch.append((req, slot, th))
            if batch:
                try:
                    self.ex.launch(key, [(req.run, slot, th) for req, slot, th in batch])
                except (RuntimeError, ValueError) as e:
                    self._fail_batch(key, [(req, slot) for req, slot, _ in batch],
                                     f"launch failed: {e}", _status_of(e))
                    continue
                self.inflight[key] = [(req, slot) for req, slot, _ in batch]

    def _in_use(self, run: int) -> bool:
        r = self.runs[run]
        return r.busy or bool(r.queue)

    def run_trace(self, requests: list, idle_sleep: float = 0.0) -> list:
        """Serve a list of requests with given arrival times (seconds from the
        start of the trace); returns them completed."""
        pending = sorted(requests, key=lambda q: q.t_arrival)
        t0 = self.clock()
        for q in pending:
            q.t_arrival += t0
        i = 0
        n = len(pending)
        while len(self.completed) < n:
            now = self.clock()
            while i < n and pending[i].t_arrival <= now:
                self.submit(pending[i])
                i += 1
            self.poll()
            self.schedule()
            if not self.inflight and i < n and not any(r.queue for r in self.runs.values()):
                wait = pending[i].t_arrival - self.clock()
                if wait > 2e-4:
                    time.sleep(min(wait - 1e-4, 1e-3))
            elif idle_sleep:
                time.sleep(idle_sleep)
        for q in pending:
            q.t_arrival -= t0
            q.t_start -= t0
            q.t_done -= t0
        return pending


STATUS_EINVAL = -1      # the library's VQE_EINVAL
STATUS_ENOMEM = -3      # the library's VQE_ENOMEM
STATUS_UNKNOWN = -4     # a failure without a library status (reported as a HIP-side error)


def _status_of(e) -> int:
    st = getattr(e, "status", None)
    return int(st) if isinstance(st, int) else STATUS_UNKNOWN


def poisson_trace(n_requests: int, rate: float, n_runs: int, seed: int) -> list:
    """Poisson arrivals at `rate` requests/s, each for a uniformly drawn run."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    runs = rng.integers(0, n_runs, size=n_requests)
    t = np.cumsum(gaps)
    return [Request(i, int(runs[i]), float(t[i])) for i in range(n_requests)]


def latency_summary(reqs: list, skip: int = 0) -> dict:
    """Latency percentiles and throughput of the completed requests after the
    first `skip` (warm-up); failed requests are counted, not timed."""
    tail = reqs[skip:]
    ok = [q for q in tail if not q.failed]
    lat = np.array([q.latency for q in ok]) * 1e3
    span = max(q.t_done for q in ok) - min(q.t_arrival for q in ok)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "p999_ms": float(np.percentile(lat, 99.9)), "mean_ms": float(lat.mean()),
            "updates_per_s": len(lat) / span, "n": int(len(lat)),
            "failed": int(len(tail) - len(ok)),
            "cold": int(sum(q.cold for q in ok))}


# ---------------------------------------------------------------------- device
class DeviceExecutor(Executor):
    """Slot groups on the GPU: one batch plan per register size."""

    def __init__(self, systems: dict, slots_per_group: int = 16, dtype: str = "c64",
                 schedules: dict | None = None, device: int = 0):
        """`systems`: run -> vqe_system.System.  `schedules`: register-size key ->
        H-product schedule, or "tuned" for the autotuner's choice for the first
        run of that size (cached, else timed here), or None for the library's
        default for that run.  With a sliced schedule each run's layout of H is
        built once when the run is admitted and slots point to it; otherwise
        every slot's plan-owned layout is sized on that first run here, so
        that binding runs of the same size later does not reallocate while
        other groups run."""
        import torch
        from . import batch as PB
        from . import binding as B
        self.torch, self.B, self.PB = torch, B, PB
        self.systems = systems                       # run -> vqe_system.System
        self.dtype = dtype
        self.keyof = {r: (s.spec.n_qubits, s.spec.n_electrons, s.spec.mapping)
                      for r, s in systems.items()}
        self.dev: dict = {}                          # run -> DeviceSystem (resident)
        self.saved: dict = {}                        # run -> host copy of psi (evicted)
        self.group: dict = {}
        self.key_fp: dict = {}
        keys = sorted(set(self.keyof.values()))
        tdt = torch.complex64 if dtype == "c64" else torch.complex128
        for key in keys:
            n_q = key[0]
            stream = torch.cuda.Stream(device=device)
            ctx = B.Context(device, stream)
            pools = PB.PoolCache(ctx)
            rep = next(s for r, s in systems.items() if self.keyof[r] == key)
            pool = pools.get(key, rep.pool, dtype)
            dim = 1 << n_q
            # placeholder binding for idle slots: an empty operator (never run)
            empty = B.csr_build_from_pauli(ctx, n_q, [], [], [], dtype=dtype)
            # one run of this size is built once up front: its device size is
            # the footprint estimate for the size, and it fixes the default
            # schedule when none is given
            rep_run = next(r for r in systems if self.keyof[r] == key)
            with torch.cuda.stream(stream):
                probe = PB.device_system(ctx, systems[rep_run], dtype, _SinglePool(pool))
            stream.synchronize()
            self.key_fp[key] = probe.H.nbytes() + dim * probe.psi.element_size()
            # the idle-slot placeholder (no terms, so vacuously real) takes the
            # representative's real flag: the slot's effective schedule then
            # equals that of the runs later bound to it
            if not probe.H.real:
                empty.desc.flags &= ~B.VQE_REAL
            if schedules == "tuned":
                from . import tune as T
                sched_k = T.schedule_for(ctx, probe, systems=[probe], value_form="any")
            elif schedules and key in schedules:
                sched_k = int(schedules[key])
            else:
                sched_k = B.default_schedule(probe.H)
            sliced = bool(sched_k & B.VQE_SPMV_SLICED)
            if sliced:
                # a run's footprint includes its layout
                lay = B.Layout(ctx, probe.H, sched_k)
                self.key_fp[key] += lay.nbytes()
                lay.close()
            sched = [sched_k] * slots_per_group
            states = []
            with torch.cuda.stream(stream):
                for _ in range(slots_per_group):
                    states.append((empty, pool, torch.zeros(dim, dtype=tdt, device="cuda")))
                plan = B.BatchPlan(ctx, states, schedules=sched, with_active=True)
                plan.active.zero_()
                # size every slot's own layout of H on the probe, then unbind
                # (a sliced schedule binds the runs' own layouts instead)
                for slot in range(slots_per_group if not sliced else 0):
                    plan.rebind(slot, probe.H, probe.pool, probe.psi)
                    plan.rebind(slot, empty, pool, states[slot][2])
            stream.synchronize()
            del probe
            pin = dict(pin_memory=True)
            # idle slots of a sliced group point to the placeholder's own
            # layout, so unbinding a run rebuilds nothing
            empty_layout = B.Layout(ctx, empty, sched_k) if sliced else None
            self.group[key] = {"ctx": ctx, "stream": stream, "plan": plan, "pool": pool,
                               "empty": empty, "empty_layout": empty_layout, "event": None,
                               "dim": dim, "sched": sched_k, "sliced": sliced,
                               "slots": slots_per_group,
                               "h_active": torch.zeros(slots_per_group, dtype=torch.int32, **pin),
                               "h_theta": torch.zeros(slots_per_group, dtype=torch.float64, **pin),
                               "h_e": torch.zeros(3 * slots_per_group, dtype=torch.float64, **pin),
                               "h_k": torch.zeros(slots_per_group, dtype=torch.int32, **pin),
                               "h_g": torch.zeros(slots_per_group, dtype=torch.float64, **pin)}
        torch.cuda.synchronize()

    # -- Executor interface
    def groups(self) -> dict:
        return {k: g["slots"] for k, g in self.group.items()}

    def run_key(self, run: int) -> tuple:
        return self.keyof[run]

    def footprint(self, run: int) -> int:
        s = self.systems[run]
        dim = 1 << s.spec.n_qubits
        # the device size once built, else the size measured for a run of the
        # same register size (plus 5%)
        if run in self.dev:
            ds = self.dev[run]
            lay = getattr(ds, "layout", None)
            return ds.H.nbytes() + dim * ds.psi.element_size() + (lay.nbytes() if lay else 0)
        return int(self.key_fp[self.keyof[run]] * 1.05)

    def fixed_bytes(self) -> int:
        total = 0
        for g in self.group.values():
            total += g["plan"].workspace_bytes() + g["pool"].nbytes()
            total += sum(t.numel() * t.element_size() for t in g["plan"].sigma) * 2
        return total

    def admit(self, run: int):
        torch = self.torch
        key = self.keyof[run]
        g = self.group[key]
        with torch.cuda.stream(g["stream"]):
            ds = self.PB.device_system(g["ctx"], self.systems[run], self.dtype,
                                       _SinglePool(g["pool"]))
            if run in self.saved:
                ds.psi.copy_(self.saved.pop(run).to(ds.psi.device))
            if g["sliced"]:
                ds.layout = self.B.Layout(g["ctx"], ds.H, g["sched"])
        g["stream"].synchronize()
        self.dev[run] = ds

    def evict(self, run: int):
        key = self.keyof[run]
        g = self.group[key]
        g["stream"].synchronize()
        self.unbind(run)
        ds = self.dev.pop(run)
        self.saved[run] = ds.psi.detach().cpu().clone()
        if getattr(ds, "layout", None) is not None:
            ds.layout.close()
        del ds
        g["stream"].synchronize()

    def launch(self, key: tuple, batch: list):
        torch = self.torch
        g = self.group[key]
        plan = g["plan"]
        bound = g.setdefault("bound", {})
        # the group's previous launch has completed (the scheduler checks), so
        # its pinned staging buffers are free to overwrite
        active = g["h_active"].numpy()
        theta = g["h_theta"].numpy()
        active[:] = 0
        for run, slot, th in batch:
            if bound.get(slot) != run:
                ds = self.dev[run]
                plan.rebind(slot, ds.H, ds.pool, ds.psi, layout=getattr(ds, "layout", None))
                bound[slot] = run
            active[slot] = 1
            theta[slot] = th
        with torch.cuda.stream(g["stream"]):
            plan.active.copy_(g["h_active"], non_blocking=True)
            plan.theta.copy_(g["h_theta"], non_blocking=True)
            plan.step(renorm=True, graph=True)
            g["h_e"].copy_(plan.energies, non_blocking=True)
            g["h_k"].copy_(plan.k, non_blocking=True)
            g["h_g"].copy_(plan.gmax, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(g["stream"])
        g["event"] = ev

    def done(self, key: tuple) -> bool:
        ev = self.group[key]["event"]
        return ev is None or ev.query()

    def results(self, key: tuple, batch: list) -> list:
        g = self.group[key]
        plan = g["plan"]
        # copied into pinned memory by the launch; its event has completed
        e = g["h_e"].numpy()[0::3]
        k = g["h_k"].numpy()
        gm = g["h_g"].numpy()
        return [(float(e[slot]), int(k[slot]), float(gm[slot])) for _, slot in batch]

    def release(self, key: tuple, slot: int):
        g = self.group[key]
        run = g.get("bound", {}).get(slot)
        if run is not None:
            self.unbind(run)

    def psi(self, run: int):
        if run in self.dev:
            return self.dev[run].psi.detach().cpu().numpy()
        return self.saved[run].numpy()

    def unbind(self, run: int):
        """Point any slot bound to `run` back at the placeholder (before eviction)."""
        for g in self.group.values():
            for slot, r in list(g.get("bound", {}).items()):
                if r == run:
                    with self.torch.cuda.stream(g["stream"]):
                        g["plan"].rebind(slot, g["empty"], g["pool"], g["plan"].states[slot][2],
                                         layout=g["empty_layout"])
                    del g["bound"][slot]


class _SinglePool:
    """PoolCache stand-in returning the slot group's pool."""

    def __init__(self, pool):
        self.pool = pool

    def get(self, key, packs, dtype):
        return self.pool


def run_sequential(ctx, systems: dict, requests: list, thetas: dict, dtype: str = "c128",
                   clock=time.perf_counter) -> list:
    """The plain single-request GPU path on the same trace: requests served one
    at a time in arrival order with the single-call entry points (energy,
    pool_gradients, vqe_select, taylor5_apply), synchronised per request; every
    run resident."""
    import torch
    with torch.cuda.stream(ctx.stream):      # torch's copies ordered with the library's work
        return _run_sequential(ctx, systems, requests, thetas, dtype, clock)


def _run_sequential(ctx, systems, requests, thetas, dtype, clock):
    import torch
    from . import batch as PB
    from . import binding as B
    pools = PB.PoolCache(ctx)
    dev = {r: PB.device_system(ctx, s, dtype, pools) for r, s in systems.items()}
    sig = {r: torch.empty_like(d.psi) for r, d in dev.items()}
    steps = collections.Counter()
    torch.cuda.synchronize()
    pending = sorted(requests, key=lambda q: q.t_arrival)
    t0 = clock()
    for q in pending:
        now = clock() - t0
        if now < q.t_arrival:
            time.sleep(q.t_arrival - now)
        q.t_start = clock() - t0
        d = dev[q.run]
        out = B.energy(ctx, d.H, d.psi, sig[q.run])
        g = B.pool_gradients(ctx, d.H, d.pool, d.psi, sig[q.run])
        k, gm = B.vqe_select(ctx, g)
        kk = int(k.cpu()[0])
        th = thetas[q.run]
        B.taylor5_apply(ctx, d.pool.ops[kk], float(th[steps[q.run] % len(th)]), d.psi,
                        renormalize=True)
        ctx.stream.synchronize()
        steps[q.run] += 1
        q.t_done = clock() - t0
        q.energy, q.selected, q.gmax = float(out.cpu()[0]), kk, float(gm.cpu()[0])
    return pending
