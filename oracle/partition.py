"""Commuting-family partition of an operator pool (Sec. III-F, Alg. 1).

TEST INFRASTRUCTURE ONLY (the oracle): plain Python, independent of the
product package.

  commutator_terms  -- [A, B] of two Pauli sums (Eq. 3) as a Pauli sum
  commutes          -- [A, B] == 0 (every combined coefficient vanishes)
  noncommutation_graph -- the complementary graph of Alg. 1: an edge (i, j)
                       iff [A_i, A_j] != 0 (full operator commutation)
  greedy_partition  -- Alg. 1: vertices by descending degree (largest
                       first), each to the lowest-indexed family holding none
                       of its neighbours, a new family when there is none
"""
from __future__ import annotations

import numpy as np


def _popcount(v: int) -> int:
    return bin(v).count("1")


def pauli_product(x1: int, z1: int, x2: int, z2: int):
    """P(x1,z1) P(x2,z2) = i^e P(x1^x2, z1^z2) with P(x,z) = i^{|x&z|} X^x Z^z;
    returns (x, z, e mod 4).  Moving Z^{z1} past X^{x2} gives (-1)^{|z1&x2|}."""
    x3, z3 = x1 ^ x2, z1 ^ z2
    e = _popcount(x1 & z1) + _popcount(x2 & z2) - _popcount(x3 & z3) + 2 * _popcount(z1 & x2)
    return x3, z3, e % 4


def anticommute(x1: int, z1: int, x2: int, z2: int) -> bool:
    """Two Pauli strings anticommute iff their symplectic product is odd."""
    return (_popcount(x1 & z2) + _popcount(z1 & x2)) % 2 == 1


def commutator_terms(a, b) -> dict:
    """[A, B] = sum over anticommuting term pairs of 2 a_s b_t P_s P_t, with
    equal strings combined: {(x, z): coefficient}."""
    out: dict = {}
    ip = [1, 1j, -1, -1j]
    for xs, zs, cs in zip(a.xmask, a.zmask, a.coeff):
        for xt, zt, ct in zip(b.xmask, b.zmask, b.coeff):
            xs_, zs_, xt_, zt_ = int(xs), int(zs), int(xt), int(zt)
            if not anticommute(xs_, zs_, xt_, zt_):
                continue
            x, z, e = pauli_product(xs_, zs_, xt_, zt_)
            out[(x, z)] = out.get((x, z), 0.0) + 2.0 * complex(cs) * complex(ct) * ip[e]
    return out


def commutes(a, b, rel_tol: float = 1e-12) -> bool:
    scale = float(np.abs(np.asarray(a.coeff)).sum() * np.abs(np.asarray(b.coeff)).sum())
    return all(abs(c) <= rel_tol * scale for c in commutator_terms(a, b).values())


def noncommutation_graph(packs) -> np.ndarray:
    """Boolean M x M adjacency of the complementary graph of Alg. 1."""
    M = len(packs)
    adj = np.zeros((M, M), dtype=bool)
    for i in range(M):
        for j in range(i + 1, M):
            if not commutes(packs[i], packs[j]):
                adj[i, j] = adj[j, i] = True
    return adj


def greedy_partition(adj: np.ndarray) -> np.ndarray:
    """Alg. 1 on a boolean adjacency matrix; ties in degree keep the canonical
    (index) order.  Returns the family index of every vertex."""
    adj = np.asarray(adj, dtype=bool)
    M = adj.shape[0]
    degree = adj.sum(axis=1)
    order = sorted(range(M), key=lambda v: (-int(degree[v]), v))
    family = np.full(M, -1, dtype=np.int64)
    members: list = []
    for v in order:
        for k, fam in enumerate(members):
            if not any(adj[v, u] for u in fam):
                family[v] = k
                fam.append(v)
                break
        else:
            family[v] = len(members)
            members.append([v])
    return family
