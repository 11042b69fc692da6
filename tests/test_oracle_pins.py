"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself.  The references are: dense
Kronecker-product Pauli matrices, fermionic operators built from their action
on occupation states (dense_ref), eigendecomposition-based exponentials, the
closed form of the truncated series for excitation generators, finite
differences, exact conservation laws, connectivity counts, and Table II.
"""
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import dense_ref as D
import vqe_system as vs
from oracle import oracle as orc


def _sys(n, ne, mapping="jw", stretched=False, seed=11, e_const=0.0):
    return vs.make_system(vs.SystemSpec(n, ne, mapping, stretched, seed, e_const))


# ---------------------------------------------------------------- CSR build (Sec. III-E)

@pytest.mark.parametrize("seed", range(6))
def test_csr_matches_kronecker_sum(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    T = int(rng.integers(1, 40))
    x = rng.integers(0, 1 << n, T).astype(np.uint64)
    z = rng.integers(0, 1 << n, T).astype(np.uint64)
    c = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    # plant an exact cancellation and a duplicate string
    x = np.concatenate([x, x[:2]])
    z = np.concatenate([z, z[:2]])
    c = np.concatenate([c, [-c[0], 0.5 * c[1]]])
    m = orc.csr_build(n, x, z, c)
    ref = D.pauli_sum_dense(n, x, z, c)
    tol = orc.default_tol(c)
    np.testing.assert_allclose(m.dense(), ref, atol=1e-15 * np.abs(c).sum())
    # canonical form: strictly ascending columns, no entry under the drop rule,
    # and every reference entry above it present
    for r in range(m.dim):
        cols = m.col[m.rowptr[r]:m.rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
    v = m.val
    assert not np.any((np.abs(v.real) <= tol) & (np.abs(v.imag) <= tol))
    big = (np.abs(ref.real) > 10 * tol) | (np.abs(ref.imag) > 10 * tol)
    assert int(big.sum()) <= m.nnz


def test_csr_drop_rule_and_empty():
    # X - X cancels exactly: an empty matrix
    m = orc.csr_build(2, [1, 1], [0, 0], [1.0, -1.0])
    assert m.nnz == 0 and np.all(m.rowptr == 0)
    m = orc.csr_build(3, [], [], [], tol=0.0)
    assert m.nnz == 0
    # identity: diagonal only
    m = orc.csr_build(3, [0], [0], [2.0])
    assert m.nnz == 8 and np.all(m.col == np.arange(8)) and np.all(m.val == 2.0)


def connectivity_nnz(n_qubits: int, e_const_zero: bool = True) -> int:
    """Entries of a generic spin-conserving two-body Hamiltonian over the full
    Fock space: per occupation row, the diagonal plus every spin-conserving
    single and double excitation.  With no constant term the vacuum diagonal
    is exactly zero."""
    m_sp = n_qubits // 2
    total = 0
    for occ in range(1 << n_qubits):
        na = bin(occ & int("01" * m_sp, 2)).count("1")
        nb = bin(occ & int("10" * m_sp, 2)).count("1")
        ha, hb = m_sp - na, m_sp - nb
        singles = na * ha + nb * hb
        doubles = comb(na, 2) * comb(ha, 2) + comb(nb, 2) * comb(hb, 2) + na * ha * nb * hb
        total += 1 + singles + doubles
    return total - (1 if e_const_zero else 0)


@pytest.mark.parametrize("n,ne", [(8, 4), (10, 4), (12, 8)])
def test_hamiltonian_nnz_connectivity(n, ne):
    H = orc.csr_from_pack(_sys(n, ne).hamiltonian)
    assert H.nnz == connectivity_nnz(n)


@pytest.mark.slow
def test_hamiltonian_nnz_connectivity_14():
    H = orc.csr_from_pack(_sys(14, 6).hamiltonian)
    assert H.nnz == connectivity_nnz(14) == 2596863


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_hamiltonian_hermitian_and_eq2(mapping):
    s = _sys(8, 4, mapping, seed=5, e_const=0.3)
    H = orc.csr_from_pack(s.hamiltonian)
    Hd = H.dense()
    # identical ordered sums on both sides of the diagonal: bit-exact Hermitian
    assert np.array_equal(Hd, Hd.conj().T)
    beta = None if mapping == "jw" else vs.encoding_matrix(mapping, 8)
    ref = D.fermion_hamiltonian(s.integrals.h, s.integrals.g, s.integrals.e_const, beta).toarray()
    np.testing.assert_allclose(Hd, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_pool_csr_structure(mapping):
    n, ne = 10, 4
    for exc, pack in zip(vs.excitation_list(n, ne), vs.pool_packs(n, ne, mapping)):
        A = orc.csr_from_pack(pack)
        assert A.nnz == (1 << (n - 1) if len(exc.occ) == 1 else 1 << (n - 3))
        assert set(np.unique(A.val)) <= {1.0 + 0j, -1.0 + 0j}
        rl = np.diff(A.rowptr)
        assert rl.max() == 1
        rows = np.nonzero(rl)[0]
        partner = A.col[A.rowptr[rows]]
        # involutive pairing: col(col(r)) = r, and anti-symmetric values
        assert np.all(A.col[A.rowptr[partner]] == rows)
        assert np.all(A.val[A.rowptr[partner]] == -A.val[A.rowptr[rows]])


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_jw_bk_permutation(mapping):
    """H_BK[beta n, beta m] = H_JW[n, m]; BK only permutes indices."""
    n, ne = 10, 4
    sj = _sys(n, ne, "jw", seed=21)
    sb = _sys(n, ne, "bk", seed=21)
    Hj = orc.csr_from_pack(sj.hamiltonian)
    Hb = orc.csr_from_pack(sb.hamiltonian)
    assert Hj.nnz == Hb.nnz
    assert sorted(np.diff(Hj.rowptr)) == sorted(np.diff(Hb.rowptr))
    P = D.encoding_permutation(vs.bk_matrix(n))
    lhs = (P @ sp.csr_matrix(Hj.dense()) @ P.T).toarray()
    np.testing.assert_allclose(Hb.dense(), lhs, atol=1e-12 * np.abs(lhs).max())


# ---------------------------------------------------------------- SpMV and Taylor (Eq. 6-8)

def test_spmv_matches_dense():
    rng = np.random.default_rng(2)
    s = _sys(8, 4, seed=2)
    H = orc.csr_from_pack(s.hamiltonian)
    x = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    np.testing.assert_allclose(orc.spmv(H, x), H.dense() @ x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(orc.spmv(H, x), D.fermion_hamiltonian(
        s.integrals.h, s.integrals.g, 0.0).toarray() @ x, atol=1e-12)
    # complex-valued matrix entries (a Pauli sum with complex coefficients)
    n, T = 6, 30
    px = rng.integers(0, 1 << n, T).astype(np.uint64)
    pz = rng.integers(0, 1 << n, T).astype(np.uint64)
    pc = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    M = orc.csr_build(n, px, pz, pc)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    np.testing.assert_allclose(orc.spmv(M, v), D.pauli_sum_dense(n, px, pz, pc) @ v, atol=1e-12)


def test_taylor_matches_dense_series_and_expm():
    rng = np.random.default_rng(4)
    n = 8
    for exc, pack in list(zip(vs.excitation_list(n, 4), vs.pool_packs(n, 4)))[::5]:
        A = orc.csr_from_pack(pack)
        Ad = D.excitation_generator(n, exc.occ, exc.vir).toarray()
        psi = rng.standard_normal(256) + 1j * rng.standard_normal(256)
        theta = float(rng.uniform(-0.5, 0.5))
        out = orc.taylor5(A, theta, psi)
        np.testing.assert_allclose(out, D.taylor5_dense(theta, Ad) @ psi, atol=1e-13)
        exact = D.expm_antihermitian(theta, Ad) @ psi
        # truncation error of the order-5 series: the sixth-order remainder
        bound = (abs(theta) ** 6 / 720) * np.linalg.norm(psi) * 1.01
        assert np.linalg.norm(out - exact) <= bound


def test_taylor_general_antihermitian_dense():
    """A generic (not pairing) anti-Hermitian Pauli sum."""
    rng = np.random.default_rng(9)
    n = 5
    T = 12
    x = rng.integers(0, 32, T).astype(np.uint64)
    z = rng.integers(0, 32, T).astype(np.uint64)
    c = 1j * rng.standard_normal(T)        # i * Hermitian Pauli = anti-Hermitian
    A = orc.csr_build(n, x, z, c)
    Ad = D.pauli_sum_dense(n, x, z, c)
    psi = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    theta = 0.37
    np.testing.assert_allclose(orc.taylor5(A, theta, psi), D.taylor5_dense(theta, Ad) @ psi,
                               atol=1e-12)
    np.testing.assert_array_equal(orc.taylor5(A, 0.0, psi), psi)


def _closed_form(theta, Apsi, A2psi, psi):
    s5 = theta - theta ** 3 / 6 + theta ** 5 / 120
    c4 = theta ** 2 / 2 - theta ** 4 / 24
    return psi + s5 * Apsi + c4 * A2psi


@pytest.mark.parametrize("n,ne", [(10, 4), (12, 8), pytest.param(14, 6, marks=pytest.mark.slow)])
def test_taylor_closed_form_excitations(n, ne):
    """For an excitation generator A^3 = -A, so the series collapses to
    psi + s5 A psi + c4 A^2 psi with s5 = t - t^3/6 + t^5/120, c4 = t^2/2 - t^4/24."""
    rng = np.random.default_rng(n)
    exc = vs.excitation_list(n, ne)
    packs = vs.pool_packs(n, ne)
    for k in (0, len(exc) - 1, len(exc) // 2):
        A = orc.csr_from_pack(packs[k])
        Asp = D.excitation_generator(n, exc[k].occ, exc[k].vir)
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        theta = float(rng.uniform(-0.1, 0.1))
        Apsi = Asp @ psi
        ref = _closed_form(theta, Apsi, Asp @ Apsi, psi)
        np.testing.assert_allclose(orc.taylor5(A, theta, psi), ref, atol=1e-14 * np.abs(psi).max())


def test_norm_growth_closed_form():
    """||T5 psi||^2 - ||psi||^2 = ||A psi||^2 ((1-c4)^2 + s5^2 - 1)
    = ||A psi||^2 (t^6/360 - t^8/960 + t^10/14400) for excitation generators."""
    n, ne = 10, 4
    rng = np.random.default_rng(1)
    exc = vs.excitation_list(n, ne)[3]
    A = orc.csr_from_pack(vs.generator_pack(exc, n))
    Asp = D.excitation_generator(n, exc.occ, exc.vir)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    for theta in (0.1, -0.7, 1.3):
        out = orc.taylor5(A, theta, psi)
        growth = np.vdot(out, out).real - np.vdot(psi, psi).real
        na = np.linalg.norm(Asp @ psi) ** 2
        poly = theta ** 6 / 360 - theta ** 8 / 960 + theta ** 10 / 14400
        # the difference of two norms of size |psi|^2 carries rounding of about
        # eps * |psi|^2, far below the O(theta^6) growth being checked
        nrm = np.vdot(psi, psi).real
        assert growth == pytest.approx(na * poly, rel=1e-6, abs=64 * 2.2e-16 * nrm)


# ---------------------------------------------------------------- energy (Eq. 1) and gradient (Eq. 5)

def test_energy_matches_dense_and_variational_bound():
    n, ne = 8, 4
    s = _sys(n, ne, seed=3)
    H = orc.csr_from_pack(s.hamiltonian)
    Hd = D.fermion_hamiltonian(s.integrals.h, s.integrals.g, 0.0).toarray()
    rng = np.random.default_rng(0)
    mask = D.sector_mask(n, ne // 2, ne // 2)
    lam0 = np.linalg.eigvalsh(Hd[np.ix_(mask, mask)])[0]
    for _ in range(3):
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[mask] = rng.standard_normal(mask.sum()) + 1j * rng.standard_normal(mask.sum())
        e, nn, im, sigma = orc.energy(H, psi)
        ref = np.vdot(psi, Hd @ psi) / np.vdot(psi, psi)
        assert e == pytest.approx(ref.real, abs=1e-12)
        assert nn == pytest.approx(np.vdot(psi, psi).real, rel=1e-14)
        assert abs(im) < 1e-10
        assert e >= lam0 - 1e-12
        np.testing.assert_allclose(sigma, Hd @ psi, atol=1e-12)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_gradient_finite_difference_and_commutator(mapping):
    n, ne = 8, 4
    s = _sys(n, ne, mapping, seed=8)
    beta = None if mapping == "jw" else vs.encoding_matrix(mapping, n)
    H = orc.csr_from_pack(s.hamiltonian)
    Hd = D.fermion_hamiltonian(s.integrals.h, s.integrals.g, 0.0, beta).toarray()
    rng = np.random.default_rng(5)
    mask = D.sector_mask(n, ne // 2, ne // 2, beta)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[mask] = rng.standard_normal(mask.sum())
    psi /= np.linalg.norm(psi)
    pool = [orc.csr_from_pack(p) for p in s.pool]
    _, _, _, sigma = orc.energy(H, psi)
    g = orc.gradients(pool, psi, sigma)
    h = 1e-4
    for j, exc in enumerate(vs.excitation_list(n, ne)):
        Ad = D.excitation_generator(n, exc.occ, exc.vir, beta).toarray()
        comm = np.vdot(psi, (Hd @ Ad - Ad @ Hd) @ psi)
        assert g[j] == pytest.approx(comm.real, abs=1e-12)
        assert abs(comm.imag) < 1e-12

        def E(t):
            ph = psi + np.sin(t) * (Ad @ psi) + (1 - np.cos(t)) * (Ad @ (Ad @ psi))
            return np.vdot(ph, Hd @ ph).real / np.vdot(ph, ph).real
        fd = (E(h) - E(-h)) / (2 * h)
        assert g[j] == pytest.approx(fd, abs=1e-7)


def test_select_tie_rule():
    assert orc.select([0.1, -0.5, 0.5, 0.2])[0] == 1
    assert orc.select([0.1, 0.5 * (1 - 1e-7), -0.5])[0] == 1
    assert orc.select([0.1, 0.5 * (1 - 1e-5), -0.5])[0] == 2
    k, gm = orc.select([0.0, 0.0])
    assert k == 0 and gm == 0.0


# ---------------------------------------------------------------- adaptive loop (Sec. III-D)

def _exact_rotation(n, exc, beta, theta, psi):
    Asp = D.excitation_generator(n, exc.occ, exc.vir, beta)
    Ap = Asp @ psi
    return psi + np.sin(theta) * Ap + (1 - np.cos(theta)) * (Asp @ Ap)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_adapt_fidelity_and_conservation(cfg):
    """Fidelity against exact evolution along the same operator/angle sequence
    exceeds 0.999999 (Abstract), amplitudes outside the (n_alpha, n_beta)
    sector stay exactly zero, and the energy obeys the variational bound."""
    specs, steps = vs.config_c1() if cfg == "c1" else vs.config_c2()
    if cfg == "c2":
        specs = [specs[1], specs[2]]        # BK-equilibrium and JW-stretched variants
    for spec in specs:
        s = vs.make_system(spec)
        n, ne = spec.n_qubits, spec.n_electrons
        beta = None if spec.mapping == "jw" else vs.encoding_matrix(spec.mapping, n)
        H = orc.csr_from_pack(s.hamiltonian)
        pool = [orc.csr_from_pack(p) for p in s.pool]
        thetas = vs.draw_thetas(spec.seed, steps)
        tr = orc.adapt_run(H, pool, vs.reference_state(s), thetas, steps)
        exc = vs.excitation_list(n, ne)
        psi = vs.reference_state(s)
        for k, t in zip(tr.selected, tr.thetas):
            psi = _exact_rotation(n, exc[k], beta, t, psi)
        assert D.fidelity(psi, tr.psi) > 0.999999
        mask = D.sector_mask(n, ne // 2, ne // 2, beta)
        assert np.all(tr.psi[~mask] == 0.0)
        assert abs(np.linalg.norm(tr.psi) - 1.0) < 1e-14
        if n <= 12:
            Hsp = D.fermion_hamiltonian(s.integrals.h, s.integrals.g, 0.0, beta)
            Hs = Hsp[mask][:, mask].toarray()
            lam0 = np.linalg.eigvalsh(Hs)[0]
            assert min(tr.energies) >= lam0 - 1e-10
            ex = (np.vdot(psi, Hsp @ psi) / np.vdot(psi, psi)).real
            assert abs(tr.energies[-1] - ex) < 1e-6


def test_jw_bk_same_trajectory_energies():
    """Mapping invariance (Sec. IV-B): along the same (k_t, theta_t) the JW and
    BK runs give the same energies."""
    n, ne, steps = 12, 8, 8
    sj = _sys(n, ne, "jw", seed=31)
    sb = _sys(n, ne, "bk", seed=31)
    Hj, Hb = orc.csr_from_pack(sj.hamiltonian), orc.csr_from_pack(sb.hamiltonian)
    pj = [orc.csr_from_pack(p) for p in sj.pool]
    pb = [orc.csr_from_pack(p) for p in sb.pool]
    th = vs.draw_thetas(31, steps)
    tj = orc.adapt_run(Hj, pj, vs.reference_state(sj), th, steps)
    tb = orc.adapt_run(Hb, pb, vs.reference_state(sb), th, steps, forced=tj.selected)
    np.testing.assert_allclose(tb.energies, tj.energies, rtol=0, atol=1e-12)
    for gj, gb in zip(tj.gradients, tb.gradients):
        np.testing.assert_allclose(gb, gj, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_csr_rows_are_rows_of_the_kronecker_sum(mapping):
    """orc_csr_rows (selected rows, any order, with repeats) gives those rows
    of the dense Kronecker-product matrix of the Pauli sum, and bit for bit
    the full builder's rows; the sampled product equals the dense product at
    those rows.  Bad rows and masks outside the register are refused."""
    s = vs.make_system(vs.SystemSpec(8, 4, mapping, False, 23), with_pool=False)
    h = s.hamiltonian
    dense = D.pauli_sum_dense(8, h.xmask, h.zmask, h.coeff)
    full = orc.csr_from_pack(h)
    rows = np.random.default_rng(24).integers(0, 256, 80)
    rows[:3] = [255, 0, 255]
    R = orc.csr_rows(h, rows)
    x = np.random.default_rng(25).standard_normal(256) + 1j * np.random.default_rng(26).standard_normal(256)
    for j, r in enumerate(rows):
        a = slice(R.rowptr[j], R.rowptr[j + 1])
        b = slice(full.rowptr[r], full.rowptr[r + 1])
        assert np.array_equal(R.col[a], full.col[b]) and np.array_equal(R.val[a], full.val[b])
        row = np.zeros(256, dtype=np.complex128)
        row[R.col[a]] = R.val[a]
        np.testing.assert_allclose(row, dense[r], rtol=0, atol=1e-15 * np.abs(h.coeff).sum())
    np.testing.assert_allclose(orc.spmv_rows(R, x), (dense @ x)[rows], rtol=0,
                               atol=1e-13 * np.abs(dense @ x).max())
    with pytest.raises(ValueError):
        orc.csr_rows(h, [256])
    bad = vs.PauliPack(8, np.array([1 << 8], dtype=np.uint64), np.array([0], dtype=np.uint64),
                       np.array([1.0 + 0j]))
    with pytest.raises(ValueError):
        orc.csr_rows(bad, [0])
