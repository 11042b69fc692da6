"""Pins of the oracle's commuting-family partition (Sec. III-F, Alg. 1).

* the Pauli product rule and the symplectic commutation test agree with
  dense 2x2 Kronecker products;
* the commutator of two Pauli sums equals the dense commutator, and the
  non-commutation graph of whole pools (JW and BK) equals the graph from
  dense commutators;
* the greedy colouring reproduces hand-worked cases and always yields
  families that commute pairwise, each vertex in the lowest family open to it.
"""
import itertools

import numpy as np
import pytest

import vqe_system as vs
from oracle import partition as P
from tests.dense_ref import pauli_string_dense, pauli_sum_dense


def test_product_rule_and_symplectic_test_match_dense():
    rng = np.random.default_rng(7)
    n = 4
    for _ in range(200):
        x1, z1, x2, z2 = (int(v) for v in rng.integers(0, 1 << n, size=4))
        A = pauli_string_dense(n, x1, z1)
        Bm = pauli_string_dense(n, x2, z2)
        x, z, e = P.pauli_product(x1, z1, x2, z2)
        np.testing.assert_allclose(A @ Bm, (1j ** e) * pauli_string_dense(n, x, z), atol=1e-14)
        anti = np.allclose(A @ Bm, -Bm @ A)
        assert P.anticommute(x1, z1, x2, z2) == anti
        assert anti != np.allclose(A @ Bm, Bm @ A)


def dense_of(pack):
    return pauli_sum_dense(pack.n_qubits, pack.xmask, pack.zmask, pack.coeff)


def test_commutator_terms_equal_dense_commutator():
    s = vs.make_system(vs.SystemSpec(8, 4, "bk", False, 41))
    n = 8
    for i, j in [(0, 1), (0, 5), (3, 9), (2, len(s.pool) - 1), (10, 20)]:
        a, b = s.pool[i], s.pool[j]
        C = dense_of(a) @ dense_of(b) - dense_of(b) @ dense_of(a)
        terms = P.commutator_terms(a, b)
        D = np.zeros_like(C)
        for (x, z), c in terms.items():
            D += c * pauli_string_dense(n, x, z)
        np.testing.assert_allclose(D, C, atol=1e-13)


@pytest.mark.parametrize("n,ne,mapping", [(4, 2, "jw"), (6, 2, "jw"), (6, 2, "bk"), (8, 4, "jw")])
def test_graph_equals_dense_commutators(n, ne, mapping):
    s = vs.make_system(vs.SystemSpec(n, ne, mapping, False, 42))
    dense = [dense_of(p) for p in s.pool]
    adj = P.noncommutation_graph(s.pool)
    for i, j in itertools.combinations(range(len(s.pool)), 2):
        C = dense[i] @ dense[j] - dense[j] @ dense[i]
        assert adj[i, j] == (np.abs(C).max() > 1e-12), (i, j)
    assert not adj.diagonal().any() and (adj == adj.T).all()


def test_greedy_hand_worked_cases():
    # complete graph K4: four families
    k4 = ~np.eye(4, dtype=bool)
    assert list(P.greedy_partition(k4)) == [0, 1, 2, 3]
    # 4-cycle 0-1-2-3-0, equal degrees: index order gives 0,1,0,1
    c4 = np.zeros((4, 4), dtype=bool)
    for a, b in [(0, 1), (1, 2), (2, 3), (3, 0)]:
        c4[a, b] = c4[b, a] = True
    assert list(P.greedy_partition(c4)) == [0, 1, 0, 1]
    # star centred at 3 (highest degree goes first), leaves share a family
    star = np.zeros((5, 5), dtype=bool)
    for leaf in (0, 1, 2, 4):
        star[3, leaf] = star[leaf, 3] = True
    assert list(P.greedy_partition(star)) == [1, 1, 1, 0, 1]
    # no edges: one family
    assert list(P.greedy_partition(np.zeros((3, 3), dtype=bool))) == [0, 0, 0]


def test_greedy_families_are_valid_and_lowest():
    rng = np.random.default_rng(3)
    for trial in range(20):
        M = int(rng.integers(2, 30))
        a = rng.random((M, M)) < rng.uniform(0.05, 0.6)
        adj = np.triu(a, 1)
        adj = adj | adj.T
        fam = P.greedy_partition(adj)
        for i, j in itertools.combinations(range(M), 2):
            if adj[i, j]:
                assert fam[i] != fam[j]
        # replay the largest-first order: each vertex took the lowest family
        # free of its already placed neighbours
        deg = adj.sum(1)
        placed = []
        for v in sorted(range(M), key=lambda v: (-deg[v], v)):
            blocked = {fam[u] for u in placed if adj[v, u]}
            assert fam[v] == min(set(range(M + 1)) - blocked)
            placed.append(v)


def test_pool_families_commute_pairwise():
    s = vs.make_system(vs.SystemSpec(8, 4, "jw", True, 43))
    fam = P.greedy_partition(P.noncommutation_graph(s.pool))
    dense = [dense_of(p) for p in s.pool]
    for k in range(fam.max() + 1):
        members = np.nonzero(fam == k)[0]
        for i, j in itertools.combinations(members, 2):
            C = dense[i] @ dense[j] - dense[j] @ dense[i]
            assert np.abs(C).max() <= 1e-12
