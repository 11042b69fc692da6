"""Line search over the selected generator's angle, in batch plans.

Along the GPU's own selections and angles, the FP64 oracle reproduces the
energies (1e-12 in FP64 storage), and at every step the GPU's angle is a
minimiser of the oracle's objective (the energy of the renormalised
fifth-order update, minimised directly by grid and Brent's method): within
1e-6 of the oracle's angle (a flat minimum fixes the angle only to about
sqrt(eps)) and with a step energy within 1e-12 of the oracle's minimum.  FP32
storage at 14 qubits within the FP32 bars.  Matrix-free pools agree with CSR
pools; graph replays agree with eager steps; generators without A^3 = -A are
refused.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2606_29692_amd import batch as PB  # noqa: E402
from paper_2606_29692_amd import binding as B  # noqa: E402

THETA_MAX = 1.0


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


def specs():
    return [vs.SystemSpec(8, 4, "jw", False, 301), vs.SystemSpec(10, 4, "bk", False, 302),
            vs.SystemSpec(12, 8, "jw", True, 303)]


def run_gpu(ctx, systems, dtype, steps, matrix_free=False, graph=False, sched=0):
    pools = PB.PoolCache(ctx, matrix_free=matrix_free)
    ds = [PB.device_system(ctx, s, dtype, pools) for s in systems]
    plan = PB.make_batch(ctx, ds, schedules=[sched] * len(ds) if sched else None)
    plan.set_line_search(THETA_MAX)
    E, K, T = [], [], []
    for t in range(steps):
        print(f"line search {dtype} mf={matrix_free} graph={graph} step {t}", flush=True)
        plan.step(renorm=True, line_search=True, graph=graph)
        E.append(host(plan.energies).reshape(-1, 3)[:, 0].copy())
        K.append(host(plan.k).copy())
        T.append(host(plan.theta).copy())
    plan.step(update=False)
    E.append(host(plan.energies).reshape(-1, 3)[:, 0].copy())
    psi = [host(d.psi).copy() for d in ds]
    plan.close()
    return np.array(E), np.array(K), np.array(T), psi


def check_against_oracle(system, E, K, T, psi_gpu, theta_tol, e_tol, min_tol):
    """The oracle follows the GPU's selections and angles (energies must
    agree), and at every step the GPU's angle minimises the oracle's step
    energy: within theta_tol of the oracle's own line search, and its energy
    within min_tol of the oracle's minimum (the minimum is flat, so angles
    agree only to about sqrt(eps); energies at them to rounding)."""
    h = orc.csr_from_pack(system.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in system.pool]
    psi = vs.reference_state(system)
    for t in range(len(K)):
        assert abs(orc.energy(h, psi)[0] - E[t]) <= e_tol
        a = pool[int(K[t])]
        th_o, e_o = orc.line_search(h, a, psi, THETA_MAX)
        e_g = orc.step_energy(h, a, psi, float(T[t]))
        print(f"  step {t}: theta gpu {T[t]:.10f} oracle {th_o:.10f}; E(gpu) - E(oracle) = {e_g - e_o:.2e}")
        assert abs(T[t] - th_o) <= theta_tol
        assert e_g <= e_o + min_tol
        psi, _ = orc.normalize(orc.taylor5(a, float(T[t]), psi))
    assert abs(orc.energy(h, psi)[0] - E[len(K)]) <= e_tol
    p = psi_gpu.astype(np.complex128)
    fid = abs(np.vdot(p, psi)) ** 2 / (np.vdot(p, p).real * np.vdot(psi, psi).real)
    return fid


def test_line_search_fp64_vs_oracle(ctx):
    sp = specs()
    systems = [vs.make_system(s) for s in sp]
    steps = 4
    E, K, T, psi = run_gpu(ctx, systems, "c128", steps)
    for i, s in enumerate(systems):
        print(f"state {i} ({sp[i].mapping}, N={sp[i].n_qubits})")
        fid = check_against_oracle(s, E[:, i], K[:, i], T[:, i], psi[i], 1e-6, 1e-12, 1e-12)
        assert fid > 1 - 1e-12
        # each step lowers the energy
        assert np.all(np.diff(E[:, i]) <= 1e-12)


def test_line_search_matrix_free_equals_csr_and_graph(ctx):
    sp = specs()
    systems = [vs.make_system(s) for s in sp]
    a = run_gpu(ctx, systems, "c128", 3, matrix_free=False, graph=False)
    b = run_gpu(ctx, systems, "c128", 3, matrix_free=True, graph=True)
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_allclose(b[2], a[2], rtol=0, atol=1e-9)
    np.testing.assert_allclose(b[0], a[0], rtol=0, atol=1e-12)
    c = run_gpu(ctx, systems, "c128", 3, matrix_free=True, graph=False)
    # graph replays equal the eager steps bit for bit
    for x, y in zip(b, c):
        if isinstance(x, list):
            for u, v in zip(x, y):
                np.testing.assert_array_equal(u, v)
        else:
            np.testing.assert_array_equal(x, y)


# the default schedule, the pipelined one with 16-bit column codes, and the
# benchmark's (the same with the real values of the real H)
@pytest.mark.parametrize("sched", [0, 32 | B.VQE_SPMV_LDS | B.VQE_SPMV_PREFETCH | B.VQE_SPMV_X16,
                                   32 | B.VQE_SPMV_LDS | B.VQE_SPMV_PREFETCH | B.VQE_SPMV_X16 |
                                   B.VQE_SPMV_REAL])
def test_line_search_fp32_14_qubits(ctx, sched):
    sp, _ = vs.config_c4(n_states=4, mixed=False)
    systems = [vs.make_system(s) for s in sp]
    steps = 2
    E, K, T, psi = run_gpu(ctx, systems, "c64", steps, matrix_free=True, graph=True, sched=sched)
    fid = check_against_oracle(systems[0], E[:, 0], K[:, 0], T[:, 0], psi[0], 1e-4, 1e-6, 1e-9)
    assert fid > 0.999999


def test_line_search_refuses_other_generators(ctx):
    n = 6
    s = vs.make_system(vs.SystemSpec(n, 2, "jw", False, 9))
    # a real symmetric pairing operator (a Pauli X string): A[r,c] A[c,r] = +1
    x_only = vs.PauliPack(n, np.array([0b000011], dtype=np.uint64), np.array([0], dtype=np.uint64),
                          np.array([1.0], dtype=np.complex128))
    pool = B.pool_from_packs(ctx, [s.pool[0], x_only], "c128")
    H = B.csr_from_pack(ctx, s.hamiltonian, "c128")
    psi = torch.zeros(1 << n, dtype=torch.complex128, device=ctx.torch_device)
    psi[s.reference_index] = 1.0
    plan = B.BatchPlan(ctx, [(H, pool, psi)])
    with pytest.raises(B.VqeError) as e:
        plan.set_line_search(THETA_MAX)
    assert e.value.status == -5
    with pytest.raises(B.VqeError):
        plan.step(line_search=True)
    plan.close()
