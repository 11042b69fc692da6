"""Pins of the input generator (integrals, Pauli algebra, JW/BK, pool).

Checked against textbook definitions (dense Pauli matrices, ladder operators
defined by their action on occupation states) and the pool sizes printed in
Table II.
"""
import json
import os

import numpy as np
import pytest

import dense_ref as D
import vqe_system as vs
from vqe_system.pauli import IPOW

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pauli_product_matches_dense():
    rng = np.random.default_rng(0)
    n = 4
    for _ in range(50):
        x1, z1, x2, z2 = (int(v) for v in rng.integers(0, 1 << n, 4))
        x3, z3, c3 = vs.multiply(x1, z1, 1.0, x2, z2, 1.0)
        lhs = D.pauli_string_dense(n, x1, z1) @ D.pauli_string_dense(n, x2, z2)
        rhs = complex(c3) * D.pauli_string_dense(n, int(x3), int(z3))
        np.testing.assert_allclose(lhs, rhs, atol=1e-15)


def test_pauli_action_rule():
    # P(x,z)|c> = i^{|x&z|} (-1)^{|z&c|} |c^x>
    n = 3
    for x in range(8):
        for z in range(8):
            P = D.pauli_string_dense(n, x, z)
            for c in range(8):
                ph = IPOW[bin(x & z).count("1") % 4] * (-1) ** bin(z & c).count("1")
                assert P[c ^ x, c] == pytest.approx(ph)


def test_labels_roundtrip():
    labels = np.array([b"XIYZ", b"IIII", b"ZZXY"])
    n, x, z = vs.from_labels(labels)
    assert n == 4
    assert list(vs.to_labels(4, x, z)) == list(labels)
    # rightmost character is qubit 0
    assert int(x[0]) == 0b1010 and int(z[0]) == 0b0011


@pytest.mark.parametrize("mapping", ["jw", "bk"])
@pytest.mark.parametrize("n", [4, 6])
def test_ladder_matches_definition(mapping, n):
    beta = vs.encoding_matrix(mapping, n)
    ref = D.annihilators(n, None if mapping == "jw" else beta)
    lx, lz, lc = vs.ladder_table(mapping, n)
    for j in range(n):
        a = D.pauli_sum_dense(n, lx[j], lz[j], lc[j])
        np.testing.assert_allclose(a, ref[j].toarray(), atol=1e-15)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_canonical_anticommutation(mapping):
    n = 6
    lx, lz, lc = vs.ladder_table(mapping, n)
    a = [D.pauli_sum_dense(n, lx[j], lz[j], lc[j]) for j in range(n)]
    eye = np.eye(1 << n)
    for i in range(n):
        for j in range(n):
            ac = a[i] @ a[j].conj().T + a[j].conj().T @ a[i]
            np.testing.assert_allclose(ac, eye if i == j else 0 * eye, atol=1e-14)
            np.testing.assert_allclose(a[i] @ a[j] + a[j] @ a[i], 0 * eye, atol=1e-14)


def test_bk_matrix_small_and_weights():
    # qubit i stores modes (i & (i+1)) .. i; for N = 4: n0, n0+n1, n2, n0+..+n3
    b = vs.bk_matrix(4)
    assert b.tolist() == [[1, 0, 0, 0], [1, 1, 0, 0], [0, 0, 1, 0], [1, 1, 1, 1]]
    for n in (8, 16):
        lx, lz, _ = vs.ladder_table("bk", n)
        w = vs.popcount(lx | lz)
        assert int(w.max()) <= int(np.ceil(np.log2(n))) + 1
        jx, jz, _ = vs.ladder_table("jw", n)
        assert int(vs.popcount(jx | jz).max()) == n  # Z string on all lower modes


def test_pool_sizes_table2():
    with open(os.path.join(GOLDEN, "table2_sizes.json")) as f:
        gold = json.load(f)
    for row in gold["rows"]:
        n, ne = row["qubits"], row["electrons"]
        assert 2 ** n == row["dim"]
        assert 4 ** n == row["elements"]
        if row.get("pool_pinned", True):
            assert vs.pool_size_formula(n, ne) == row["pool"]
            assert len(vs.excitation_list(n, ne)) == row["pool"]


@pytest.mark.parametrize("n,ne,m", [(8, 4, 26), (10, 4, 54), (12, 6, 117), (16, 6, 315), (16, 8, 360)])
def test_pool_size_formula(n, ne, m):
    assert vs.pool_size_formula(n, ne) == m == len(vs.excitation_list(n, ne))


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_generators_match_definition(mapping):
    n, ne = 6, 2
    beta = None if mapping == "jw" else vs.encoding_matrix(mapping, n)
    for exc, pack in zip(vs.excitation_list(n, ne), vs.pool_packs(n, ne, mapping)):
        A = D.pauli_sum_dense(n, pack.xmask, pack.zmask, pack.coeff)
        ref = D.excitation_generator(n, exc.occ, exc.vir, beta).toarray()
        np.testing.assert_allclose(A, ref, atol=1e-15)
        np.testing.assert_allclose(A, -A.conj().T, atol=0)
        assert np.all(pack.coeff.real == 0.0)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
@pytest.mark.parametrize("stretched", [False, True])
def test_hamiltonian_pack_matches_eq2(mapping, stretched):
    n_orb = 3
    ints = vs.gen_integrals(n_orb, seed=7, stretched=stretched, e_const=0.25)
    pack = vs.hamiltonian_pack(ints, mapping)
    Hp = D.pauli_sum_dense(2 * n_orb, pack.xmask, pack.zmask, pack.coeff)
    beta = None if mapping == "jw" else vs.encoding_matrix(mapping, 2 * n_orb)
    Hf = D.fermion_hamiltonian(ints.h, ints.g, ints.e_const, beta).toarray()
    scale = np.abs(Hf).max()
    np.testing.assert_allclose(Hp, Hf, atol=1e-13 * scale)
    assert np.all(pack.coeff.imag == 0.0)


def test_integrals_symmetry_and_recipe():
    ints = vs.gen_integrals(5, seed=3)
    h, g = ints.h, ints.g
    np.testing.assert_array_equal(h, h.T)
    assert np.all(np.diff(np.diag(h)) >= 0)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        np.testing.assert_array_equal(g, g.transpose(perm))
    st = vs.gen_integrals(5, seed=3, stretched=True)
    d0, d1 = np.diag(h), np.diag(st.h)
    np.testing.assert_allclose(d1 - d1[0], (d0 - d0[0]) / 5.0, atol=1e-15)
    # same seed, same draw; different seed, different draw
    np.testing.assert_array_equal(vs.gen_integrals(5, seed=3).g, g)
    assert not np.array_equal(vs.gen_integrals(5, seed=4).g, g)


def test_reference_index():
    s = vs.make_system(vs.SystemSpec(8, 4, "jw", False, 1))
    assert s.reference_index == 0b1111
    sb = vs.make_system(vs.SystemSpec(8, 4, "bk", False, 1))
    assert sb.reference_index == vs.encode_bits(vs.bk_matrix(8), 0b1111)
