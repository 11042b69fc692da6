"""Registers larger than LDS at 18 and 20 qubits: the blocked column-tiled H
product (per (row block, column tile) slabs, tile-local 16-bit codes,
accumulators in LDS) and its sliced form (each slab's rows sorted into
64-row slices, one row per lane), FP32 storage against the FP64 oracle.

* 18 qubits (262,144 rows, about 1.2e8 entries per H): sigma = H psi on every
  row and the energy (Eq. 1) for JW and BK systems with seeded complex start
  states, at several sub-group widths; and two adaptive steps (Eq. 5 screen,
  selection, Eq. 6-8 update, renormalisation) along the GPU's selections
  against orc.adapt_run (FP32 bars: |dE| < 1e-6, |dg| < 1e-5, fidelity >
  0.999999).
* 20 qubits (1,048,576 rows, about 7e8 entries): the oracle builds only the
  rows it needs (orc.csr_rows): sigma on every row of the particle sector
  (H conserves the particle numbers, so H psi lives there), the energy from
  those rows, and sigma exactly zero at sampled rows outside the sector.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2606_29692_amd import batch as PB  # noqa: E402
from paper_2606_29692_amd import binding as B  # noqa: E402

P = B.VQE_SPMV_LDS | B.VQE_SPMV_PREFETCH


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
def systems18():
    specs = [vs.SystemSpec(18, 8, m, False, vs.system_seed(180, i)) for i, m in enumerate(["jw", "bk"])]
    out = []
    for s in specs:
        sy = vs.make_system(s, with_pool=False)
        print(f"oracle CSR of the 18-qubit {s.mapping} Hamiltonian", flush=True)
        out.append((sy, orc.csr_from_pack(sy.hamiltonian)))
    return out


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


S = B.VQE_SPMV_LDS | B.VQE_SPMV_SLICED


@pytest.mark.parametrize("sched", [8 | P, 16 | P, 32 | P, 16 | P | B.VQE_SPMV_DEEP,
                                   8 | P | B.VQE_SPMV_DEEP, 8 | P | B.VQE_SPMV_DEEP | B.VQE_SPMV_X16,
                                   64 | P | B.VQE_SPMV_X16, 4 | P, 4 | P | B.VQE_SPMV_X16,
                                   2 | S, 4 | S, 8 | S, 2 | S | B.VQE_SPMV_DEEP])
def test_blocked_18_qubits_sigma_energy(ctx, systems18, sched):
    pools = PB.PoolCache(ctx, matrix_free=True)
    ds, psis = [], []
    for sy, _ in systems18:
        sy.pool = vs.shared_pool(18, 8, sy.spec.mapping)
        d = PB.device_system(ctx, sy, "c64", pools)
        p = vs.complex_start_state(sy).astype(np.complex64)
        d.psi.copy_(torch.from_numpy(p))
        ds.append(d)
        psis.append(p.astype(np.complex128))
    plan = PB.make_batch(ctx, ds, schedules=[sched] * len(ds))
    print(f"18 qubits, schedule {sched}: step", flush=True)
    plan.step(update=False)
    e = host(plan.energies).reshape(-1, 3)
    for i, (sy, oH) in enumerate(systems18):
        e_o, n2_o, _, sg_o = orc.energy(oH, psis[i])
        sg = host(plan.sigma[i]).astype(np.complex128)
        ref = sg_o - ds[i].H.diag_shift * psis[i]
        err = np.linalg.norm(sg - ref) / np.linalg.norm(ref)
        print(f"  {sy.spec.mapping}: |dE| {abs(e[i, 0] - e_o):.2e}, sigma rel err {err:.2e}")
        assert abs(e[i, 0] - e_o) < 1e-6
        assert abs(e[i, 1] - n2_o) < 1e-6
        assert err < 2e-6
    plan.close()


def test_blocked_18_qubits_adaptive_steps(ctx, systems18):
    sy, oH = systems18[0]
    sy.pool = vs.shared_pool(18, 8, "jw")
    pools = PB.PoolCache(ctx, matrix_free=True)
    d = PB.device_system(ctx, sy, "c64", pools)
    p0 = vs.complex_start_state(sy).astype(np.complex64)
    d.psi.copy_(torch.from_numpy(p0))
    plan = PB.make_batch(ctx, [d], schedules=[16 | P])
    steps = 2
    th = vs.draw_thetas(sy.spec.seed, steps)
    E, K, G = [], [], []
    for t in range(steps):
        print(f"18 qubits adaptive step {t}", flush=True)
        plan.theta.copy_(torch.tensor([th[t]], dtype=torch.float64))
        plan.step(renorm=True, graph=True)
        E.append(float(host(plan.energies)[0]))
        K.append(int(host(plan.k)[0]))
        G.append(host(plan.gradients(0)).copy())
    plan.step(update=False)
    E.append(float(host(plan.energies)[0]))
    psi = host(d.psi).astype(np.complex128)
    plan.close()
    print("oracle pool CSRs (560 generators)", flush=True)
    opool = [orc.csr_from_pack(q) for q in sy.pool]
    tr = orc.adapt_run(oH, opool, p0.astype(np.complex128), th, steps, forced=K)
    de = np.abs(np.array(E) - np.array(tr.energies)).max()
    dg = max(np.abs(G[t] - tr.gradients[t]).max() for t in range(steps))
    fid = abs(np.vdot(psi, tr.psi)) ** 2 / (np.vdot(psi, psi).real * np.vdot(tr.psi, tr.psi).real)
    print(f"18 qubits, {steps} steps: max|dE| {de:.2e}, max|dg| {dg:.2e}, 1 - F {1 - fid:.2e}")
    assert de < 1e-6 and dg < 1e-5 and fid > 0.999999
    for t in range(steps):
        g_o = tr.gradients[t]
        assert abs(g_o[K[t]]) >= np.abs(g_o).max() * (1 - 1e-5)


@pytest.mark.parametrize("sched", [16 | P, 2 | S, 2 | S | B.VQE_SPMV_DEEP])
def test_blocked_20_qubits_sector_rows(ctx, sched):
    sy = vs.make_system(vs.SystemSpec(20, 10, "jw", False, vs.system_seed(200, 0)), with_pool=False)
    sy.pool = vs.shared_pool(20, 10, "jw")
    pools = PB.PoolCache(ctx, matrix_free=True)
    print("20 qubits: device build", flush=True)
    d = PB.device_system(ctx, sy, "c64", pools)
    p = vs.complex_start_state(sy).astype(np.complex64)
    d.psi.copy_(torch.from_numpy(p))
    plan = PB.make_batch(ctx, [d], schedules=[sched])
    print(f"20 qubits, schedule {sched}: step", flush=True)
    plan.step(update=False)
    e = host(plan.energies)[:3].copy()
    sg = host(plan.sigma[0]).astype(np.complex128)
    shift = d.H.diag_shift
    plan.close()
    del d, plan
    psi = p.astype(np.complex128)
    sector = vs.sector_indices(sy)
    print(f"oracle rows of the sector ({sector.size})", flush=True)
    R = orc.csr_rows(sy.hamiltonian, sector)
    sg_o = orc.spmv_rows(R, psi)
    ref = sg_o - shift * psi[sector]
    err = np.linalg.norm(sg[sector] - ref) / np.linalg.norm(ref)
    n2 = float(np.vdot(psi[sector], psi[sector]).real)
    e_o = float(np.vdot(psi[sector], sg_o).real) / n2
    print(f"20 qubits: sector sigma rel err {err:.2e}, |dE| {abs(e[0] - e_o):.2e}")
    assert err < 2e-6
    assert abs(e[0] - e_o) < 1e-6 and abs(e[1] - n2) < 1e-6
    outside = np.setdiff1d(np.random.default_rng(201).integers(0, 1 << 20, 20000), sector)
    assert np.all(sg[outside] == 0.0)
