"""Second-quantised Hamiltonian (Eq. 2) and excitation pool, mapped to Pauli sums.

Spin-orbital m = 2p + sigma (sigma = 0 for alpha), stored in bit m of the
occupation vector.  The Hamiltonian

    H = sum_ij h_ij a_i^+ a_j + 1/2 sum_ijkl h_ijkl a_i^+ a_j^+ a_l a_k

uses h_ij = h[p_i, p_j] delta(s_i, s_j) and h_ijkl = <ij|kl> = (p_i p_k | p_j p_l)
delta(s_i, s_k) delta(s_j, s_l).  Its Pauli form (Eq. 3) is obtained by
multiplying out the ladder-operator expansions of the chosen encoding.  The
structure of that expansion (which strings, with which phase, from which
integral) depends only on (N, mapping), so it is built once and re-used for
every seed: a new Hamiltonian costs one weighted bincount.

The pool holds the spin-conserving single and double excitations out of the
aufbau reference (lowest n_e spin-orbitals occupied), as anti-Hermitian
generators A = T - T^+ with unit coefficient, in canonical order: singles
(i, a) then doubles (i, j, a, b) with i<j and a<b, each lexicographic.  Its
size reproduces the pool sizes of Table II (92 at 12 qubits / 8 electrons,
204 at 14 qubits / 6 electrons).
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache
from itertools import combinations

import numpy as np

from .encoding import ladder_table
from .integrals import Integrals
from .pauli import IPOW, merge, popcount


def _product_expand(mapping: str, n: int, ops: np.ndarray, dag: np.ndarray):
    """Multiply out products of ladder operators.

    ``ops`` is (n_prod, f) mode indices, ``dag`` (f,) booleans (creator or not).
    Returns x, z, c of shape (n_prod, 2**f): the Pauli expansion of each product.
    """
    lx, lz, lc = ladder_table(mapping, n)
    n_prod, f = ops.shape
    x = np.zeros((n_prod, 1), dtype=np.uint64)
    z = np.zeros((n_prod, 1), dtype=np.uint64)
    c = np.ones((n_prod, 1), dtype=np.complex128)
    for k in range(f):
        m = ops[:, k]
        fx = lx[m]                # (n_prod, 2)
        fz = lz[m]
        fc = np.conj(lc[m]) if dag[k] else lc[m]
        x1 = np.repeat(x, 2, axis=1)
        z1 = np.repeat(z, 2, axis=1)
        c1 = np.repeat(c, 2, axis=1)
        x2 = np.tile(fx, (1, x.shape[1]))
        z2 = np.tile(fz, (1, x.shape[1]))
        c2 = np.tile(fc, (1, x.shape[1]))
        x3 = x1 ^ x2
        z3 = z1 ^ z2
        e = popcount(x1 & z1) + popcount(x2 & z2) - popcount(x3 & z3) + 2 * popcount(z1 & x2)
        x, z, c = x3, z3, c1 * c2 * IPOW[e % 4]
    return x, z, c


@dataclass(frozen=True)
class _Expansion:
    key: np.ndarray      # unique (x<<32|z) keys, sorted
    inv: np.ndarray      # product-term -> unique key index
    w: np.ndarray        # complex weight of each product term
    src: np.ndarray      # index into the flattened integral vector


@lru_cache(maxsize=None)
def _hamiltonian_expansion(mapping: str, n_qubits: int) -> _Expansion:
    n = n_qubits
    if n % 2:
        raise ValueError("spin-orbital registers have an even number of qubits")
    n_orb = n // 2
    spin = np.arange(n) % 2
    orb = np.arange(n) // 2
    # one-body a_i^+ a_j, same spin
    i1, j1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i1, j1 = i1.ravel(), j1.ravel()
    sel = spin[i1] == spin[j1]
    i1, j1 = i1[sel], j1[sel]
    src1 = orb[i1] * n_orb + orb[j1]                     # into h.ravel()
    ops1 = np.stack([i1, j1], axis=1)
    x1, z1, c1 = _product_expand(mapping, n, ops1, np.array([True, False]))
    # two-body 1/2 h_ijkl a_i^+ a_j^+ a_l a_k, s_i = s_k, s_j = s_l, i != j, k != l
    g = np.indices((n, n, n, n)).reshape(4, -1)
    i2, j2, k2, l2 = g
    sel = (spin[i2] == spin[k2]) & (spin[j2] == spin[l2]) & (i2 != j2) & (k2 != l2)
    i2, j2, k2, l2 = i2[sel], j2[sel], k2[sel], l2[sel]
    # (p_i p_k | p_j p_l) flattened, offset past the one-body block
    src2 = n_orb * n_orb + (((orb[i2] * n_orb + orb[k2]) * n_orb + orb[j2]) * n_orb + orb[l2])
    ops2 = np.stack([i2, j2, l2, k2], axis=1)
    x2, z2, c2 = _product_expand(mapping, n, ops2, np.array([True, True, False, False]))
    c2 = 0.5 * c2
    x = np.concatenate([x1.ravel(), x2.ravel()])
    z = np.concatenate([z1.ravel(), z2.ravel()])
    w = np.concatenate([c1.ravel(), c2.ravel()])
    src = np.concatenate([np.repeat(src1, x1.shape[1]), np.repeat(src2, x2.shape[1])])
    key = (x << np.uint64(32)) | z
    uk, inv = np.unique(key, return_inverse=True)
    return _Expansion(key=uk, inv=inv, w=w, src=src)


@dataclass(frozen=True)
class PauliPack:
    """Contiguous Pauli-sum buffer: operator = sum_t coeff[t] P(xmask[t], zmask[t]).

    This is the data structure the C-ABI's CSR builder consumes (the
    fixed-width label buffer of the vectorized pool layout, Sec. III-E, held as
    bit masks; :meth:`labels` gives the character form)."""
    n_qubits: int
    xmask: np.ndarray    # uint64[T]
    zmask: np.ndarray    # uint64[T]
    coeff: np.ndarray    # complex128[T]

    @property
    def n_terms(self) -> int:
        return int(self.xmask.size)

    def labels(self) -> np.ndarray:
        from .pauli import to_labels
        return to_labels(self.n_qubits, self.xmask, self.zmask)


def hamiltonian_pack(ints: Integrals, mapping: str = "jw",
                     rel_drop: float = 1e-13) -> PauliPack:
    """Pauli sum of Eq. 2 under the given mapping (real coefficients, Eq. 3).

    Strings whose merged coefficient is below rel_drop * max|c| are rounding
    residue of exact cancellations and are removed; the imaginary parts, which
    vanish exactly for a Hermitian operator, are zeroed after a check.
    """
    n = 2 * ints.n_orb
    ex = _hamiltonian_expansion(mapping, n)
    vals = np.concatenate([ints.h.ravel(), ints.g.ravel()])
    contrib = ex.w * vals[ex.src]
    re = np.bincount(ex.inv, weights=contrib.real, minlength=ex.key.size)
    im = np.bincount(ex.inv, weights=contrib.imag, minlength=ex.key.size)
    x = ex.key >> np.uint64(32)
    z = ex.key & np.uint64(0xFFFFFFFF)
    scale = max(np.abs(re).max(), 1e-300)
    if np.abs(im).max() > 1e-10 * scale:
        raise AssertionError("Hamiltonian Pauli coefficients are not real")
    if ints.e_const != 0.0:
        at0 = np.nonzero((x == 0) & (z == 0))[0]
        re[at0] += ints.e_const
    keep = np.abs(re) > rel_drop * scale
    return PauliPack(n, x[keep].copy(), z[keep].copy(), re[keep].astype(np.complex128))


def reference_occupation(n_electrons: int) -> int:
    """Aufbau reference: the lowest n_e spin-orbitals occupied."""
    return (1 << n_electrons) - 1


@dataclass(frozen=True)
class Excitation:
    occ: tuple           # annihilated spin-orbitals (i,) or (i, j), ascending
    vir: tuple           # created spin-orbitals (a,) or (a, b), ascending


def excitation_list(n_qubits: int, n_electrons: int) -> list[Excitation]:
    spin = [m % 2 for m in range(n_qubits)]
    occ = list(range(n_electrons))
    vir = list(range(n_electrons, n_qubits))
    singles = [Excitation((i,), (a,)) for i in occ for a in vir if spin[i] == spin[a]]
    doubles = []
    for (i, j) in combinations(occ, 2):
        for (a, b) in combinations(vir, 2):
            if spin[i] + spin[j] == spin[a] + spin[b]:
                doubles.append(Excitation((i, j), (a, b)))
    return singles + doubles


def pool_size_formula(n_qubits: int, n_electrons: int) -> int:
    o = n_electrons // 2
    v = n_qubits // 2 - o
    c2 = lambda k: k * (k - 1) // 2
    return 2 * o * v + 2 * c2(o) * c2(v) + (o * v) ** 2


def generator_pack(exc: Excitation, n_qubits: int, mapping: str = "jw") -> PauliPack:
    """A = T - T^+ for T = a_a^+ a_i (single) or a_a^+ a_b^+ a_j a_i (double)."""
    if len(exc.occ) == 1:
        ops = np.array([[exc.vir[0], exc.occ[0]]])
        dag = np.array([True, False])
    else:
        i, j = exc.occ
        a, b = exc.vir
        ops = np.array([[a, b, j, i]])
        dag = np.array([True, True, False, False])
    x, z, c = _product_expand(mapping, n_qubits, ops, dag)
    # (c P)^+ = conj(c) P, so T - T^+ has coefficients c - conj(c) = 2i Im(c);
    # these are sums of exact dyadic fractions, so cancellation is exact.
    x, z, c = merge(x, z, c - np.conj(c), drop_below=0.0)
    return PauliPack(n_qubits, x, z, (1j * c.imag).astype(np.complex128))


def pool_packs(n_qubits: int, n_electrons: int, mapping: str = "jw") -> list[PauliPack]:
    return [generator_pack(e, n_qubits, mapping) for e in excitation_list(n_qubits, n_electrons)]
