"""Column-tiled H product (states larger than LDS) in batch plans.

FP64 storage at 14 qubits (256 KiB state: two 128 KiB column tiles) against
the oracle to 1e-12 along forced trajectories; FP32 storage at 16 qubits
(four tiles) against the oracle within the FP32 bars; a slot rebound to
another Hamiltonian recomputes its tile bounds (or its sliced slabs); the
sliced tiles of a sparse operator at 17 and 21 qubits (blocks that reach two
or three tiles, part masks in two windows) against the oracle on every row.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2606_29692_amd import batch as PB  # noqa: E402
from paper_2606_29692_amd import binding as B  # noqa: E402

SCHED = 32 | B.VQE_SPMV_LDS | B.VQE_SPMV_PREFETCH
# the same tile passes reading 16-bit column codes (col ^ row)
SCHED_X16 = SCHED | B.VQE_SPMV_X16
# and the real parts of the values (every Hamiltonian here is real)
SCHED_R = SCHED_X16 | B.VQE_SPMV_REAL
# one row per lane, each (row block, column tile) slab sorted and sliced
SCHED_S = 2 | B.VQE_SPMV_LDS | B.VQE_SPMV_SLICED
SCHED_S4 = 4 | B.VQE_SPMV_LDS | B.VQE_SPMV_SLICED
# and the next column tile's loads in flight while a tile is multiplied
SCHED_SD = SCHED_S | B.VQE_SPMV_DEEP


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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run(ctx, systems, dtype, steps, matrix_free, sched=SCHED):
    pools = PB.PoolCache(ctx, matrix_free=matrix_free)
    ds = [PB.device_system(ctx, s, dtype, pools) for s in systems]
    plan = PB.make_batch(ctx, ds, schedules=[sched] * len(ds))
    thetas = np.stack([vs.draw_thetas(s.spec.seed, steps) for s in systems])
    E, K, G = [], [], []
    for t in range(steps):
        print(f"tiled {dtype} step {t}", flush=True)
        plan.theta.copy_(torch.from_numpy(thetas[:, t]))
        plan.step(renorm=True, graph=True)
        E.append(host(plan.energies).reshape(-1, 3)[:, 0].copy())
        K.append(host(plan.k).copy())
        G.append([host(plan.gradients(i)).copy() for i in range(len(ds))])
    plan.step(update=False)
    E.append(host(plan.energies).reshape(-1, 3)[:, 0].copy())
    psi = [host(d.psi).copy() for d in ds]
    plan.close()
    return np.array(E), np.array(K), G, psi, thetas


def oracle_run(system, thetas, K):
    return orc.adapt_run(orc.csr_from_pack(system.hamiltonian), [orc.csr_from_pack(p) for p in system.pool],
                         vs.reference_state(system), thetas, len(K), forced=K)


@pytest.mark.parametrize("matrix_free,sched", [(False, SCHED), (True, SCHED), (True, SCHED_X16),
                                                (True, SCHED_R), (True, SCHED_S), (False, SCHED_S4),
                                                (True, SCHED_SD)])
def test_tiled_fp64_14_qubits(ctx, matrix_free, sched):
    specs = [vs.SystemSpec(14, 6, m, False, vs.system_seed(60, i)) for i, m in enumerate(["jw", "bk"])]
    systems = [vs.make_system(s) for s in specs]
    E, K, G, psi, th = run(ctx, systems, "c128", 2, matrix_free, sched)
    for i, s in enumerate(systems):
        tr = oracle_run(s, th[i], K[:, i])
        np.testing.assert_allclose(E[:, i], tr.energies, rtol=0, atol=1e-12 * 10)
        for t in range(2):
            g_o = tr.gradients[t]
            np.testing.assert_allclose(G[t][i], g_o, rtol=0, atol=1e-12 * max(1, np.abs(g_o).max()))
        assert np.linalg.norm(psi[i] - tr.psi) <= 1e-12 * np.linalg.norm(tr.psi)


@pytest.mark.parametrize("sched", [SCHED, SCHED_X16, SCHED_R, SCHED_S, SCHED_S4, SCHED_SD])
def test_tiled_fp32_16_qubits(ctx, sched):
    specs = [vs.SystemSpec(16, 8, "jw", False, vs.system_seed(61, i)) for i in range(2)]
    systems = [vs.make_system(s) for s in specs]
    E, K, G, psi, th = run(ctx, systems, "c64", 1, True, sched)
    tr = oracle_run(systems[0], th[0], K[:, 0])
    de = np.abs(E[:, 0] - np.array(tr.energies)).max()
    dg = np.abs(G[0][0] - tr.gradients[0]).max()
    p = psi[0].astype(np.complex128)
    fid = abs(np.vdot(p, tr.psi)) ** 2 / (np.vdot(p, p).real * np.vdot(tr.psi, tr.psi).real)
    print(f"16 qubits: max|dE| {de:.2e}, max|dg| {dg:.2e}, 1 - F {1 - fid:.2e}")
    assert de < 1e-6 and dg < 1e-5 and fid > 0.999999


@pytest.mark.parametrize("sched", [SCHED, SCHED_X16, SCHED_R, SCHED_S, SCHED_SD])
def test_tiled_rebind(ctx, sched):
    """Slot 0 rebound to another Hamiltonian of the same size: its tile
    bounds are rebuilt, and the energy matches that system's own plan."""
    specs = [vs.SystemSpec(14, 6, "jw", False, vs.system_seed(62, i)) for i in range(2)]
    systems = [vs.make_system(s) for s in specs]
    pools = PB.PoolCache(ctx, matrix_free=True)
    a, b = (PB.device_system(ctx, s, "c128", pools) for s in systems)
    plan = PB.make_batch(ctx, [a], schedules=[sched])
    plan.rebind(0, b.H, b.pool, b.psi)
    plan.step(update=False)
    e_rebound = host(plan.energies)[:3].copy()
    own = PB.make_batch(ctx, [b], schedules=[sched])
    own.step(update=False)
    np.testing.assert_array_equal(e_rebound, host(own.energies)[:3])
    plan.close()
    own.close()


@pytest.mark.parametrize("dtype,n", [("c128", 14), ("c64", 16)])
def test_tiled_real_values_complex_state(ctx, dtype, n):
    """Column-tiled real-value schedule (tiles twice as wide, real parts in
    storage precision) on a complex state: every tile runs as two half-width
    complex passes; and on a real state; sigma (of the stored, shifted
    operator) and the energy against the oracle for both, and the schedules
    with and without real values agree."""
    s = vs.make_system(vs.SystemSpec(n, vs.ELECTRONS[n], "jw", False, 170 + n))
    oH = orc.csr_from_pack(s.hamiltonian)
    pools = PB.PoolCache(ctx, matrix_free=True)
    rng = np.random.default_rng(n)
    tol = 1e-12 if dtype == "c128" else 2e-6
    for complex_ in (True, False):
        v = rng.standard_normal(1 << n) + (1j * rng.standard_normal(1 << n) if complex_ else 0)
        v = (v / np.linalg.norm(v)).astype(np.complex128)
        sig = {}
        for sched in (SCHED_X16, SCHED_R):
            d = PB.device_system(ctx, s, dtype, pools)
            d.psi.copy_(torch.from_numpy(v))
            plan = PB.make_batch(ctx, [d], schedules=[sched])
            plan.step(update=False)
            e = host(plan.energies)[0]
            sig[sched] = host(plan.sigma[0]).astype(np.complex128)
            vin = host(d.psi).astype(np.complex128)
            e_o, _, _, sg_o = orc.energy(oH, vin)
            # the stored operator is H - shift I (FP32 storage), so sigma is
            sg_o = sg_o - d.H.diag_shift * vin
            err = np.linalg.norm(sig[sched] - sg_o) / np.linalg.norm(sg_o)
            print(f"{dtype} N={n} complex={complex_} sched={sched}: |dE| {abs(e - e_o):.2e}, "
                  f"sigma rel err {err:.2e}")
            assert abs(e - e_o) <= tol * max(1.0, abs(e_o))
            assert err <= tol
            plan.close()
        d = np.linalg.norm(sig[SCHED_R] - sig[SCHED_X16]) / np.linalg.norm(sig[SCHED_X16])
        assert d <= tol


def _sparse_pack(n):
    """Four Pauli strings on n qubits: Z on qubit 3 (diagonal), X0 X(n-1),
    X(n-1) X(n-2) (a flip of the two top qubits only, so a row block's other
    tile lies far from its own) and Y5 Y(n-3)."""
    x = [0, 1 | 1 << (n - 1), 1 << (n - 1) | 1 << (n - 2), 1 << 5 | 1 << (n - 3)]
    z = [1 << 3, 0, 0, 1 << 5 | 1 << (n - 3)]
    c = [-0.3, 0.7, 0.5, 0.2]
    return vs.PauliPack(n, np.array(x, dtype=np.uint64), np.array(z, dtype=np.uint64),
                        np.array(c, dtype=np.complex128))


@pytest.mark.parametrize("n_q", [17, 21])
@pytest.mark.parametrize("sched", [SCHED_S, SCHED_SD])
def test_sliced_tiles_of_a_sparse_operator(ctx, n_q, sched):
    """The sliced column-tiled product of an operator whose row blocks reach
    only two or three of the column tiles, and few 16 KiB parts of them (at
    21 qubits the 128 tiles span two windows of 64 part masks, and a block's
    far tile lies in the other window): sigma on every row and the energy
    against the oracle, FP32 storage."""
    pack = _sparse_pack(n_q)
    H = B.csr_from_pack(ctx, pack, "c64")
    gen = vs.PauliPack(n_q, np.array([3], dtype=np.uint64), np.array([0], dtype=np.uint64),
                       np.array([1j], dtype=np.complex128))
    pool = B.MatrixFreePool([gen], "c64")
    rng = np.random.default_rng(n_q)
    v = rng.standard_normal(1 << n_q) + 1j * rng.standard_normal(1 << n_q)
    v /= np.linalg.norm(v)
    psi = torch.from_numpy(v.astype(np.complex64)).to(ctx.torch_device)
    print(f"{n_q} qubits, schedule {sched}: plan", flush=True)
    plan = B.BatchPlan(ctx, [(H, pool, psi)], schedules=[sched])
    plan.step(update=False)
    e = host(plan.energies)[:3].copy()
    sg = host(plan.sigma[0]).astype(np.complex128)
    plan.close()
    vin = host(psi).astype(np.complex128)
    R = orc.csr_rows(pack, np.arange(1 << n_q))
    ref = orc.spmv_rows(R, vin)
    err = np.linalg.norm(sg - ref) / np.linalg.norm(ref)
    n2 = float(np.vdot(vin, vin).real)
    e_o = float(np.vdot(vin, ref).real) / n2
    print(f"  sigma rel err {err:.2e}, |dE| {abs(e[0] - e_o):.2e}")
    assert err < 2e-6
    assert abs(e[0] - e_o) < 1e-6 and abs(e[1] - n2) < 1e-6
