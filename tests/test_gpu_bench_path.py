"""The benchmark's exact call against the FP64 oracle, for every state.

64 independent 14-qubit states (7 orbitals, 6 electrons, JW), FP32 storage,
matrix-free pool (no pool CSR), the tuned H-product schedule, whole-step graph
replay, renormalisation, no line search: three adaptive steps (Eq. 5 screen,
Sec. III-D selection, Eq. 6-8 update) and the final energy (Eq. 1).

Two value forms, as the benchmark runs them:
  * complex: the interleaved complex values of H (a schedule without the
    real-value option) and states started from seeded complex states of their
    particle sector, so the H product and the screen run in complex arithmetic
    (the step flag that sends every state to the row-tiled screen);
  * real: the real-value specialisation (the real parts of a real H in the
    row-padded layout) on real states from the reference.
Every state's energies, all 204 gradients and its final state are compared
with orc.adapt_run along the GPU's own selections (FP32 bars: |dE| < 1e-6 Ha,
max|dg| < 1e-5, fidelity > 0.999999); each selection must be the oracle's, or
a near tie within the FP32 gradient error; amplitudes outside the particle
sector stay exactly zero.  The complex form also runs for eight states under
the BK mapping.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2606_29692_amd import batch as PB  # noqa: E402
from paper_2606_29692_amd import binding as B  # noqa: E402
from paper_2606_29692_amd import tune as T  # noqa: E402

STEPS = 3


@pytest.fixture(scope="module")
def ctx():
    prev = torch.cuda.current_stream()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    c = B.Context(0, stream)
    yield c
    torch.cuda.synchronize()
    c.close()
    torch.cuda.set_stream(prev)


@pytest.fixture(scope="module")
def workload():
    specs, _ = vs.config_c4(n_states=64, mixed=False)
    systems = [vs.make_system(s) for s in specs]
    opool = [orc.csr_from_pack(p) for p in systems[0].pool]
    return specs, systems, opool


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("form", ["complex", "real"])
def test_bench_call_all_states_vs_oracle(ctx, workload, form):
    specs, systems, opool = workload
    pools = PB.PoolCache(ctx, matrix_free=True)
    ds = [PB.device_system(ctx, s, "c64", pools) for s in systems]
    sched = T.schedule_for(ctx, ds[0], systems=ds, value_form="complex" if form == "complex" else "any")
    print(f"bench path, {form} form: schedule {sched}", flush=True)
    if form == "complex":
        assert not sched & B.VQE_SPMV_REAL
        psi0 = [vs.complex_start_state(s).astype(np.complex64) for s in systems]
        for d, p in zip(ds, psi0):
            d.psi.copy_(torch.from_numpy(p))
    else:
        assert sched & B.VQE_SPMV_REAL and all(d.H.real for d in ds)
        psi0 = [vs.reference_state(s).astype(np.complex64) for s in systems]
    plan = PB.make_batch(ctx, ds, schedules=[sched] * len(ds))
    thetas = np.stack([vs.draw_thetas(s.seed, STEPS) for s in specs])
    E = np.zeros((STEPS + 1, 64))
    K = np.zeros((STEPS, 64), dtype=np.int64)
    G = np.zeros((STEPS, 64, 204))
    for t in range(STEPS):
        plan.theta.copy_(torch.from_numpy(thetas[:, t]))
        plan.step(renorm=True, graph=True, tiled_screen=form == "complex")
        E[t] = host(plan.energies).reshape(-1, 3)[:, 0]
        K[t] = host(plan.k)
        G[t] = host(plan.g).reshape(64, 204)
        print(f"  step {t} done", flush=True)
    plan.step(update=False)
    E[STEPS] = host(plan.energies).reshape(-1, 3)[:, 0]
    psi_gpu = [host(d.psi).astype(np.complex128) for d in ds]
    plan.close()

    worst = {"dE": 0.0, "dg": 0.0, "1-F": 0.0}
    agree = 0
    for i, s in enumerate(systems):
        if form == "complex":
            assert np.count_nonzero(psi0[i].imag) > 1000
        oH = orc.csr_from_pack(s.hamiltonian)
        tr = orc.adapt_run(oH, opool, psi0[i].astype(np.complex128), thetas[i], STEPS,
                           forced=K[:, i])
        de = np.abs(E[:, i] - np.array(tr.energies)).max()
        dg = max(np.abs(G[t, i] - tr.gradients[t]).max() for t in range(STEPS))
        p = psi_gpu[i]
        fid = abs(np.vdot(p, tr.psi)) ** 2 / (np.vdot(p, p).real * np.vdot(tr.psi, tr.psi).real)
        worst["dE"] = max(worst["dE"], de)
        worst["dg"] = max(worst["dg"], dg)
        worst["1-F"] = max(worst["1-F"], 1 - fid)
        assert de < 1e-6, (i, de)
        assert dg < 1e-5, (i, dg)
        assert fid > 0.999999, (i, fid)
        for t in range(STEPS):
            g_o = tr.gradients[t]
            k_o, gm_o = orc.select(g_o)
            if K[t, i] == k_o:
                agree += 1
            else:
                assert abs(g_o[K[t, i]]) >= gm_o * (1 - 1e-5), (i, t, K[t, i], k_o)
        outside = np.ones(s.dim, dtype=bool)
        outside[vs.sector_indices(s)] = False
        assert np.all(p[outside] == 0.0)
    print(f"{form} form, 64 states x {STEPS} steps: max|dE| {worst['dE']:.2e} Ha, max|dg| "
          f"{worst['dg']:.2e}, max 1-F {worst['1-F']:.2e}, selections equal to the oracle's "
          f"{agree}/{64 * STEPS}")


def test_bench_call_bk_states_vs_oracle(ctx):
    """The complex form's call under the BK mapping (`bench.py --mapping bk`),
    eight states: BK generators' own tile bits form more distinct sets than
    the shared cover the screen takes, so this runs the cover's sets."""
    n = 8
    specs = [vs.SystemSpec(14, vs.ELECTRONS[14], "bk", False, vs.system_seed(44, i)) for i in range(n)]
    systems = [vs.make_system(s) for s in specs]
    opool = [orc.csr_from_pack(p) for p in systems[0].pool]
    pools = PB.PoolCache(ctx, matrix_free=True)
    ds = [PB.device_system(ctx, s, "c64", pools) for s in systems]
    sched = T.schedule_for(ctx, ds[0], systems=ds, value_form="complex")
    print(f"BK bench path: schedule {sched}", flush=True)
    assert not sched & B.VQE_SPMV_REAL
    psi0 = [vs.complex_start_state(s).astype(np.complex64) for s in systems]
    for d, p in zip(ds, psi0):
        d.psi.copy_(torch.from_numpy(p))
    plan = PB.make_batch(ctx, ds, schedules=[sched] * n)
    thetas = np.stack([vs.draw_thetas(s.seed, STEPS) for s in specs])
    E = np.zeros((STEPS + 1, n))
    K = np.zeros((STEPS, n), dtype=np.int64)
    G = np.zeros((STEPS, n, len(opool)))
    for t in range(STEPS):
        plan.theta.copy_(torch.from_numpy(thetas[:, t]))
        plan.step(renorm=True, graph=True, tiled_screen=True)
        E[t] = host(plan.energies).reshape(-1, 3)[:, 0]
        K[t] = host(plan.k)
        G[t] = host(plan.g).reshape(n, -1)
        print(f"  step {t} done", flush=True)
    plan.step(update=False)
    E[STEPS] = host(plan.energies).reshape(-1, 3)[:, 0]
    psi_gpu = [host(d.psi).astype(np.complex128) for d in ds]
    plan.close()
    for i, s in enumerate(systems):
        assert np.count_nonzero(psi0[i].imag) > 1000
        oH = orc.csr_from_pack(s.hamiltonian)
        tr = orc.adapt_run(oH, opool, psi0[i].astype(np.complex128), thetas[i], STEPS, forced=K[:, i])
        de = np.abs(E[:, i] - np.array(tr.energies)).max()
        dg = max(np.abs(G[t, i] - tr.gradients[t]).max() for t in range(STEPS))
        p = psi_gpu[i]
        fid = abs(np.vdot(p, tr.psi)) ** 2 / (np.vdot(p, p).real * np.vdot(tr.psi, tr.psi).real)
        print(f"BK state {i}: max|dE| {de:.2e}, max|dg| {dg:.2e}, 1-F {1 - fid:.2e}", flush=True)
        assert de < 1e-6 and dg < 1e-5 and fid > 0.999999, (i, de, dg, fid)
        for t in range(STEPS):
            g_o = tr.gradients[t]
            assert abs(g_o[K[t, i]]) >= np.abs(g_o).max() * (1 - 1e-5), (i, t)


def test_tiled_screen_flag(ctx, workload):
    """The step flag that sends every state to the row-tiled screen: on
    complex states the same gradients bit for bit as the plan's default
    screen (which runs the same row tiles for them from inside its launch);
    on real states the same gradients to the rounding of FP64 sums."""
    specs, systems, _ = workload
    pools = PB.PoolCache(ctx, matrix_free=True)
    sub = systems[:8]
    ds = [PB.device_system(ctx, s, "c64", pools) for s in sub]
    for i, (d, s) in enumerate(zip(ds, sub)):
        if i % 2:
            d.psi.copy_(torch.from_numpy(vs.complex_start_state(s).astype(np.complex64)))
    plan = PB.make_batch(ctx, ds, schedules=[18976] * len(ds))
    plan.step(update=False)
    g0 = host(plan.g).reshape(len(ds), -1).copy()
    plan.step(update=False, tiled_screen=True, graph=True)
    g1 = host(plan.g).reshape(len(ds), -1).copy()
    for i in range(len(ds)):
        if i % 2:
            np.testing.assert_array_equal(g1[i], g0[i])
        else:
            np.testing.assert_allclose(g1[i], g0[i], rtol=0, atol=1e-12 * max(1.0, np.abs(g0[i]).max()))
    plan.close()
