"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Bars: CSR structure and FP64 values bit-exact (the builder's sums are ordered
like the oracle's); FP64 states, energies and gradients within 1e-12
relative; FP32-storage path: fidelity > 0.999999 and |dE| < 1e-6 Ha.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2606_29692_amd as P  # noqa: E402
from paper_2606_29692_amd import binding as B  # noqa: E402

TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = P.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda").to(dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_csr_equal(d, o, values=True):
    rp = host(d.rowptr).astype(np.int64)
    np.testing.assert_array_equal(rp, o.rowptr)
    n = o.nnz
    assert d.nnz == n
    np.testing.assert_array_equal(host(d.col)[:n], o.col)
    if values:
        v = host(d.val)[:n]
        # bit-exact: compare the raw float64 words
        np.testing.assert_array_equal(v.view(np.uint64), o.val.view(np.uint64))


def rand_state(rng, dim):
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    return v / np.linalg.norm(v)


def diag_entry(o, r):
    """H[r, r] of an oracle CSR (the FP64 reference value for the shift)."""
    row = slice(o.rowptr[r], o.rowptr[r + 1])
    return float(o.val[row][o.col[row] == r][0].real)


def sys_(n, ne, mapping="jw", seed=3, stretched=False):
    return vs.make_system(vs.SystemSpec(n, ne, mapping, stretched, seed))


# ------------------------------------------------------------------ CSR build
@pytest.mark.parametrize("seed", range(8))
def test_csr_random_pauli_bit_exact(ctx, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 9))
    T = int(rng.integers(1, 300))
    x = rng.integers(0, 1 << n, T).astype(np.uint64)
    z = rng.integers(0, 1 << n, T).astype(np.uint64)
    c = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    c[: T // 3] = np.round(c[: T // 3], 1)          # exact cancellations become likely
    x = np.concatenate([x, x[:5]])
    z = np.concatenate([z, z[:5]])
    c = np.concatenate([c, -c[:5]])
    print(f"csr random seed={seed} n={n} T={x.size}", flush=True)
    o = orc.csr_build(n, x, z, c)
    d = B.csr_build_from_pauli(ctx, n, x, z, c)
    assert_csr_equal(d, o)


@pytest.mark.parametrize("n,ne,mapping", [(8, 4, "jw"), (8, 4, "bk"), (12, 8, "jw"),
                                          (12, 8, "bk"), (14, 6, "jw")])
def test_csr_hamiltonian_and_pool_bit_exact(ctx, n, ne, mapping):
    s = sys_(n, ne, mapping)
    print(f"csr H n={n} {mapping}", flush=True)
    o = orc.csr_from_pack(s.hamiltonian)
    d = B.csr_from_pack(ctx, s.hamiltonian)
    assert_csr_equal(d, o)
    assert not d.pairing
    for k in (0, len(s.pool) // 2, len(s.pool) - 1):
        od = orc.csr_from_pack(s.pool[k])
        dd = B.csr_from_pack(ctx, s.pool[k])
        assert_csr_equal(dd, od)
        assert dd.pairing


def test_csr_edge_cases(ctx):
    # empty sum, a single identity term, a cancelling pair, one qubit
    d = B.csr_build_from_pauli(ctx, 3, [], [], [])
    assert d.nnz == 0 and np.all(host(d.rowptr) == 0)
    d = B.csr_build_from_pauli(ctx, 3, [0], [0], [2.5])
    o = orc.csr_build(3, [0], [0], [2.5])
    assert_csr_equal(d, o)
    d = B.csr_build_from_pauli(ctx, 2, [1, 1], [0, 0], [1.0, -1.0])
    assert d.nnz == 0
    d = B.csr_build_from_pauli(ctx, 1, [1, 1, 0], [1, 0, 1], [0.5, 0.25j, -1.0])
    o = orc.csr_build(1, [1, 1, 0], [1, 0, 1], [0.5, 0.25j, -1.0])
    assert_csr_equal(d, o)


def test_csr_c64_shift(ctx):
    s = sys_(10, 4)
    o = orc.csr_from_pack(s.hamiltonian)
    shift = diag_entry(o, s.reference_index)
    d = B.csr_from_pack(ctx, s.hamiltonian, dtype="c64", diag_shift=shift)
    assert d.diag_shift == shift
    rp = host(d.rowptr).astype(np.int64)
    col = host(d.col)[: d.nnz]
    val = host(d.val)[: d.nnz]
    od = o.dense()
    for r in range(o.dim):
        cols = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0)
        expect = set(o.col[o.rowptr[r]:o.rowptr[r + 1]].tolist()) | {r}
        assert set(cols.tolist()) == expect
        want = od[r, cols] - shift * (cols == r)
        np.testing.assert_array_equal(val[rp[r]:rp[r + 1]], want.astype(np.complex64))


def test_csr_errors(ctx):
    with pytest.raises(B.VqeError) as e:
        B.csr_build_from_pauli(ctx, 3, [8], [0], [1.0])        # mask bit >= n_qubits
    assert e.value.status == B.VQE_EINVAL
    with pytest.raises(B.VqeError):
        B.csr_build_from_pauli(ctx, 0, [0], [0], [1.0])
    with pytest.raises(B.VqeError):
        B.csr_build_from_pauli(ctx, 2, [0], [0], [np.nan])
    with pytest.raises(B.VqeError):
        B.csr_build_from_pauli(ctx, 2, [0], [0], [1.0], dtype="c128", diag_shift=1.0)


# ------------------------------------------------------------------ energy and gradients
@pytest.mark.parametrize("n,ne,mapping", [(8, 4, "jw"), (12, 8, "bk"), (14, 6, "jw")])
def test_energy_and_gradients_fp64(ctx, n, ne, mapping):
    s = sys_(n, ne, mapping, seed=9)
    rng = np.random.default_rng(n)
    H = B.csr_from_pack(ctx, s.hamiltonian)
    oH = orc.csr_from_pack(s.hamiltonian)
    pool = B.pool_from_packs(ctx, s.pool)
    opool = [orc.csr_from_pack(p) for p in s.pool]
    for psi in (vs.reference_state(s), rand_state(rng, s.dim)):
        print(f"energy n={n} {mapping}", flush=True)
        e_o, n2_o, im_o, sig_o = orc.energy(oH, psi)
        g_o = orc.gradients(opool, psi, sig_o)
        p = dev(psi)
        sigma = torch.empty_like(p)
        out = host(B.energy(ctx, H, p, sigma))
        assert abs(out[0] - e_o) <= TOL * max(1.0, abs(e_o))
        assert abs(out[1] - n2_o) <= TOL * n2_o
        assert abs(out[2] - im_o) <= TOL * max(1.0, abs(e_o))
        sg = host(sigma)
        assert np.linalg.norm(sg - sig_o) <= TOL * max(1.0, np.linalg.norm(sig_o))
        gs = max(1.0, np.abs(g_o).max())
        g1 = host(B.pool_gradients(ctx, H, pool, p, sigma))
        np.testing.assert_allclose(g1, g_o, rtol=0, atol=TOL * gs)
        g2 = host(B.pool_gradients(ctx, H, pool, p, None))
        np.testing.assert_array_equal(g1, g2)
        k, gm = B.vqe_select(ctx, torch.from_numpy(g1).cuda())
        ko, gmo = orc.select(g1)
        assert int(host(k)[0]) == ko and float(host(gm)[0]) == gmo


def test_select_ties(ctx):
    g = torch.tensor([0.3, -0.9, 0.9 * (1 - 1e-7), 0.9, 0.1], dtype=torch.float64, device="cuda")
    k, gm = B.vqe_select(ctx, g)
    assert int(host(k)[0]) == 1 and float(host(gm)[0]) == 0.9
    g = torch.tensor([0.0] * 70 + [-2.0], dtype=torch.float64, device="cuda")
    k, _ = B.vqe_select(ctx, g)
    assert int(host(k)[0]) == 70


# ------------------------------------------------------------------ Taylor update
@pytest.mark.parametrize("n,ne,mapping", [(8, 4, "jw"), (12, 8, "bk"), (14, 6, "jw")])
def test_taylor_pairing_fp64(ctx, n, ne, mapping):
    s = sys_(n, ne, mapping)
    rng = np.random.default_rng(7)
    for k in (0, len(s.pool) - 1):
        A = B.csr_from_pack(ctx, s.pool[k])
        oA = orc.csr_from_pack(s.pool[k])
        assert A.pairing
        psi = rand_state(rng, s.dim)
        theta = float(rng.uniform(-0.5, 0.5))
        print(f"taylor pair n={n} k={k}", flush=True)
        raw = orc.taylor5(oA, theta, psi)
        p = dev(psi)
        n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
        B.taylor5_apply(ctx, A, theta, p, renormalize=False, norm2_out=n2)
        got = host(p)
        assert np.linalg.norm(got - raw) <= TOL * np.linalg.norm(raw)
        assert abs(host(n2)[0] - np.vdot(raw, raw).real) <= TOL
        p = dev(psi)
        B.taylor5_apply(ctx, A, theta, p, renormalize=True)
        want, _ = orc.normalize(raw)
        assert np.linalg.norm(host(p) - want) <= TOL


@pytest.mark.parametrize("n,T", [(6, 20), (10, 150)])
def test_taylor_generic_single_workgroup(ctx, n, T):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 1 << n, T).astype(np.uint64)
    z = rng.integers(0, 1 << n, T).astype(np.uint64)
    c = 1j * rng.standard_normal(T) * 0.3           # i * Hermitian strings: anti-Hermitian
    A = B.csr_build_from_pauli(ctx, n, x, z, c)
    oA = orc.csr_build(n, x, z, c)
    assert not A.pairing and A.nnz <= 1 << 18
    psi = rand_state(rng, 1 << n)
    raw = orc.taylor5(oA, 0.21, psi)
    p = dev(psi)
    B.taylor5_apply(ctx, A, 0.21, p, renormalize=False)
    assert np.linalg.norm(host(p) - raw) <= TOL * np.linalg.norm(raw)


def test_taylor_generic_chained(ctx):
    """A large non-pairing generator (i H at 14 qubits, 2.6e6 entries) takes the
    five-launch path."""
    s = sys_(14, 6)
    pack = s.hamiltonian
    A = B.csr_build_from_pauli(ctx, 14, pack.xmask, pack.zmask, 1j * pack.coeff * 0.05)
    oA = orc.csr_build(14, pack.xmask, pack.zmask, 1j * pack.coeff * 0.05)
    assert A.nnz > 1 << 18
    rng = np.random.default_rng(1)
    psi = rand_state(rng, 1 << 14)
    raw = orc.taylor5(oA, 0.1, psi)
    p = dev(psi)
    B.taylor5_apply(ctx, A, 0.1, p, renormalize=False)
    assert np.linalg.norm(host(p) - raw) <= TOL * np.linalg.norm(raw)


def test_taylor_errors(ctx):
    s = sys_(8, 4)
    A = B.csr_from_pack(ctx, s.pool[0])
    p = dev(vs.reference_state(s))
    with pytest.raises(B.VqeError) as e:
        B.taylor5_apply(ctx, A, float("nan"), p)
    assert e.value.status == B.VQE_EINVAL


# ------------------------------------------------------------------ adaptive runs
def run_gpu_single(ctx, s, thetas, steps, forced=None, dtype="c128", shift=0.0):
    """The plain single-request path: one C-ABI call per stage, per step."""
    H = B.csr_from_pack(ctx, s.hamiltonian, dtype=dtype, diag_shift=shift)
    pool = B.pool_from_packs(ctx, s.pool, dtype=dtype)
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    p = dev(vs.reference_state(s), tdt)
    sigma = torch.empty_like(p)
    es, gs, ks = [], [], []
    for t in range(steps):
        out = B.energy(ctx, H, p, sigma)
        g = B.pool_gradients(ctx, H, pool, p, sigma)
        k, _ = B.vqe_select(ctx, g)
        kk = int(host(k)[0]) if forced is None else int(forced[t])
        es.append(float(host(out)[0]))
        gs.append(host(g))
        ks.append(kk)
        B.taylor5_apply(ctx, pool.ops[kk], float(thetas[t]), p, renormalize=True)
    es.append(float(host(B.energy(ctx, H, p, sigma))[0]))
    return es, gs, ks, host(p).astype(np.complex128)


@pytest.mark.parametrize("which", ["c1", "c2-jw", "c2-bk", "c2-jw-stretched", "c2-bk-stretched"])
def test_adapt_trajectory_fp64(ctx, which):
    if which == "c1":
        specs, steps = vs.config_c1()
        spec = specs[0]
    else:
        specs, steps = vs.config_c2()
        m = "bk" if "bk" in which else "jw"
        spec = [x for x in specs if x.mapping == m and x.stretched == ("stretched" in which)][0]
    s = vs.make_system(spec)
    th = vs.draw_thetas(spec.seed, steps)
    print(f"adapt {which}", flush=True)
    tr = orc.adapt_run(orc.csr_from_pack(s.hamiltonian), [orc.csr_from_pack(p) for p in s.pool],
                       vs.reference_state(s), th, steps)
    es, gs, ks, psi = run_gpu_single(ctx, s, th, steps, forced=tr.selected)
    for t in range(steps):
        assert abs(es[t] - tr.energies[t]) <= TOL * max(1.0, abs(tr.energies[t]))
        gsc = max(1.0, np.abs(tr.gradients[t]).max())
        np.testing.assert_allclose(gs[t], tr.gradients[t], rtol=0, atol=TOL * gsc)
    assert abs(es[-1] - tr.energies[-1]) <= TOL * max(1.0, abs(tr.energies[-1]))
    assert np.linalg.norm(psi - tr.psi) <= TOL
    # the GPU's own selection agrees with the oracle's along the shared path
    es2, _, ks2, _ = run_gpu_single(ctx, s, th, steps)
    assert ks2 == tr.selected


def test_fp32_storage_c3(ctx):
    """FP32 state and CSR values, FP64 reductions, 30 updates at 14 qubits,
    against the FP64 oracle along the same operator sequence."""
    specs, steps = vs.config_c3()
    spec = specs[0]
    s = vs.make_system(spec)
    th = vs.draw_thetas(spec.seed, steps)
    oH = orc.csr_from_pack(s.hamiltonian)
    tr = orc.adapt_run(oH, [orc.csr_from_pack(p) for p in s.pool], vs.reference_state(s), th, steps)
    shift = diag_entry(oH, s.reference_index)
    print("fp32 c3", flush=True)
    es, gs, ks, psi = run_gpu_single(ctx, s, th, steps, forced=tr.selected, dtype="c64",
                                     shift=shift)
    de = max(abs(a - b) for a, b in zip(es, tr.energies))
    dg = max(np.abs(a - b).max() for a, b in zip(gs, tr.gradients))
    fid = abs(np.vdot(psi, tr.psi)) ** 2 / (np.vdot(psi, psi).real * np.vdot(tr.psi, tr.psi).real)
    print(f"fp32 c3: max|dE|={de:.3e} max|dg|={dg:.3e} 1-F={1 - fid:.3e}")
    assert de < 1e-6
    assert fid > 0.999999
    assert dg < 1e-5
