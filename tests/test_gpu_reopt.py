"""Re-optimisation of every angle of the adaptive ansatz (cyclic coordinate
line search) in batch plans, against the oracle.

* FP64 storage (JW and BK, 8-12 qubits, CSR and matrix-free pools): the
  oracle's ansatz energy at the GPU's final angles equals the GPU's energy
  (1e-12) and the GPU's state is the oracle's ansatz state at those angles
  (fidelity 1 - 1e-12); at every visit of the sweep the GPU's angle is a
  minimiser of the oracle's one-angle energy (within 1e-12 of the oracle's
  minimum); CSR and matrix-free pools give the same angles;
* adaptive runs on the GPU with line search and re-optimisation reach the
  exact ground energy of the reference's particle sector at 6 qubits;
* FP32 storage at 14 qubits within the FP32 bars;
* argument errors and generators without A^3 = -A are refused.
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


def run_gpu(ctx, systems, dtype, steps, sweeps, matrix_free=False, reopt_each_step=False, sched=0):
    """ADAPT steps with line search on the GPU, recording the history; then
    (or after each step) one re-optimisation.  Returns the angles before the
    final re-optimisation, the final angles, the selections, the energies
    after it and the final states."""
    pools = PB.PoolCache(ctx, matrix_free=matrix_free)
    ds = [PB.device_system(ctx, s, dtype, pools) for s in systems]
    plan = PB.make_batch(ctx, ds, schedules=[sched] * len(ds) if sched else None)
    plan.set_line_search(THETA_MAX)
    hist = PB.AnsatzHistory(plan, steps)
    e_out = torch.zeros(plan.B, dtype=torch.float64, device=ctx.torch_device)
    before = None
    for t in range(steps):
        print(f"reopt {dtype} mf={matrix_free} step {t}", flush=True)
        plan.step(renorm=True, line_search=True)
        hist.record()
        if reopt_each_step or t == steps - 1:
            before = host(hist.thetas).copy()
            hist.reoptimize(sweeps, THETA_MAX, e_out)
    after = host(hist.thetas).copy()
    ks = host(hist.ks).copy()
    e = host(e_out).copy()
    psi = [host(d.psi).copy() for d in ds]
    plan.step(update=False)
    e_next = host(plan.energies).reshape(-1, 3)[:, 0].copy()
    plan.close()
    return before, after, ks, e, psi, e_next


def specs():
    return [vs.SystemSpec(8, 4, "jw", False, 401), vs.SystemSpec(10, 4, "bk", False, 402),
            vs.SystemSpec(12, 8, "jw", True, 403)]


def oracle_parts(system):
    h = orc.csr_from_pack(system.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in system.pool]
    return h, pool, vs.reference_state(system)


def test_reopt_fp64_vs_oracle(ctx):
    sp = specs()
    systems = [vs.make_system(s) for s in sp]
    steps = 3
    before, after, ks, e, psi, e_next = run_gpu(ctx, systems, "c128", steps, sweeps=1)
    for i, s in enumerate(systems):
        h, pool, ref = oracle_parts(s)
        k = ks[i]
        e_o = orc.ansatz_energy(h, pool, ref, k, after[i])
        print(f"state {i} ({sp[i].mapping}, N={sp[i].n_qubits}): ks {list(k)} angles "
              f"{before[i]} -> {after[i]}; E gpu {e[i]:.12f} oracle {e_o:.12f}")
        assert abs(e[i] - e_o) <= 1e-12 * max(1.0, abs(e_o))
        assert abs(e_next[i] - e_o) <= 1e-12 * max(1.0, abs(e_o))
        phi = orc.ansatz_state(pool, ref, k, after[i])
        fid = abs(np.vdot(psi[i], phi)) ** 2 / (np.vdot(psi[i], psi[i]).real * np.vdot(phi, phi).real)
        assert fid > 1 - 1e-12
        # the sweep: visit m saw the new angles before m and the old ones after
        assert e_o <= orc.ansatz_energy(h, pool, ref, k, before[i]) + 1e-13
        for m in range(steps):
            cur = np.concatenate([after[i][:m], before[i][m:]])

            def f(t, m=m, cur=cur):
                trial = cur.copy()
                trial[m] = t
                return orc.ansatz_energy(h, pool, ref, k, trial)

            t_o, f_o = orc.minimise_angle(f, THETA_MAX, 201)
            print(f"  visit {m}: angle gpu {after[i][m]:.10f} oracle {t_o:.10f}; "
                  f"E(gpu) - E(oracle) = {f(after[i][m]) - f_o:.2e}")
            assert f(after[i][m]) <= f_o + 1e-12
            assert abs(after[i][m] - t_o) <= 1e-6


def test_reopt_matrix_free_equals_csr(ctx):
    systems = [vs.make_system(s) for s in specs()]
    a = run_gpu(ctx, systems, "c128", 3, sweeps=2, matrix_free=False, reopt_each_step=True)
    b = run_gpu(ctx, systems, "c128", 3, sweeps=2, matrix_free=True, reopt_each_step=True)
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_allclose(b[1], a[1], rtol=0, atol=1e-9)
    np.testing.assert_allclose(b[3], a[3], rtol=0, atol=1e-12)


def test_adapt_with_reopt_reaches_sector_ground_state(ctx):
    n = 6
    s = vs.make_system(vs.SystemSpec(n, 2, "jw", False, 35))
    amask = int("01" * (n // 2), 2)
    bmask = amask << 1
    r = s.reference_index
    na, nb = bin(r & amask).count("1"), bin(r & bmask).count("1")
    idx = [c for c in range(1 << n)
           if bin(c & amask).count("1") == na and bin(c & bmask).count("1") == nb]
    H = orc.csr_from_pack(s.hamiltonian).dense()
    e_exact = np.linalg.eigvalsh(H[np.ix_(idx, idx)]).min()
    _, after, ks, e, psi, e_next = run_gpu(ctx, [s], "c128", 10, sweeps=1, matrix_free=True,
                                           reopt_each_step=True)
    print(f"6 qubits: E - E_exact = {e_next[0] - e_exact:.3e} after 10 steps, ks {list(ks[0])}")
    assert e_next[0] - e_exact < 1e-9
    assert e_next[0] >= e_exact - 1e-12


# the default schedule, the pipelined one with 16-bit column codes, and the
# benchmark's (the same with the real values of the real H)
@pytest.mark.parametrize("sched", [0, 32 | B.VQE_SPMV_LDS | B.VQE_SPMV_PREFETCH | B.VQE_SPMV_X16,
                                   32 | B.VQE_SPMV_LDS | B.VQE_SPMV_PREFETCH | B.VQE_SPMV_X16 |
                                   B.VQE_SPMV_REAL])
def test_reopt_fp32_14_qubits(ctx, sched):
    sp, _ = vs.config_c4(n_states=2, mixed=False)
    systems = [vs.make_system(s) for s in sp]
    before, after, ks, e, psi, e_next = run_gpu(ctx, systems, "c64", 3, sweeps=1,
                                                matrix_free=True, sched=sched)
    for i, s in enumerate(systems):
        h, pool, ref = oracle_parts(s)
        e_o = orc.ansatz_energy(h, pool, ref, ks[i], after[i])
        e_b = orc.ansatz_energy(h, pool, ref, ks[i], before[i])
        phi = orc.ansatz_state(pool, ref, ks[i], after[i])
        p = psi[i].astype(np.complex128)
        fid = abs(np.vdot(p, phi)) ** 2 / (np.vdot(p, p).real * np.vdot(phi, phi).real)
        print(f"fp32 14q state {i}: |dE| = {abs(e_next[i] - e_o):.2e}, 1-F = {1 - fid:.2e}, "
              f"E drop by re-optimisation {e_b - e_o:.3e}")
        assert abs(e_next[i] - e_o) < 1e-6
        assert abs(e[i] - e_o) < 1e-6
        assert fid > 0.999999
        assert e_o <= e_b + 1e-9


def test_reopt_errors(ctx):
    n = 6
    s = vs.make_system(vs.SystemSpec(n, 2, "jw", False, 9))
    pools = PB.PoolCache(ctx)
    d = PB.device_system(ctx, s, "c128", pools)
    plan = PB.make_batch(ctx, [d])
    hist = PB.AnsatzHistory(plan, 2)
    with pytest.raises(ValueError):
        plan.reoptimize(hist.ks, hist.thetas, 3, hist.refs)
    # the C entry point checks n <= ld on its own
    ptrs = (B.C.c_void_p * 1)(hist.refs[0].data_ptr())
    rc = B.lib().vqe_batch_reoptimize(plan.handle, hist.ks.data_ptr(), hist.thetas.data_ptr(), 2,
                                      3, ptrs, 1, 1.0, None)
    assert rc == -1
    rc = B.lib().vqe_batch_reoptimize(plan.handle, hist.ks.data_ptr(), hist.thetas.data_ptr(), 2,
                                      1, ptrs, 1, 0.0, None)
    assert rc == -1
    plan.close()
    # a real symmetric pairing operator (A[r,c] A[c,r] = +1) is refused
    x_only = vs.PauliPack(n, np.array([0b000011], dtype=np.uint64), np.array([0], dtype=np.uint64),
                          np.array([1.0], dtype=np.complex128))
    pool = B.pool_from_packs(ctx, [s.pool[0], x_only], "c128")
    H = B.csr_from_pack(ctx, s.hamiltonian, "c128")
    psi = torch.zeros(1 << n, dtype=torch.complex128, device=ctx.torch_device)
    psi[s.reference_index] = 1.0
    plan = B.BatchPlan(ctx, [(H, pool, psi)])
    ks = torch.zeros((1, 1), dtype=torch.int32, device=ctx.torch_device)
    th = torch.zeros((1, 1), dtype=torch.float64, device=ctx.torch_device)
    with pytest.raises(B.VqeError) as e:
        plan.reoptimize(ks, th, 1, [psi.clone()])
    assert e.value.status == -5
    plan.close()
