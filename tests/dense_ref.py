"""Textbook dense/sparse constructions used to pin the oracle.

Nothing here calls the oracle or the HIP path.  Each routine is the plain
definition of the object it builds:
  * Pauli strings as Kronecker products of the 2x2 Pauli matrices;
  * fermionic ladder operators from their action on occupation states;
  * the Bravyi-Kitaev ladders as the basis permutation P_beta applied to the
    Jordan-Wigner ones;
  * the second-quantised Hamiltonian (Eq. 2) assembled from those ladders;
  * matrix exponentials through an eigendecomposition.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

I2 = np.eye(2, dtype=np.complex128)
X2 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z2 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def pauli_string_dense(n: int, x: int, z: int) -> np.ndarray:
    """Kronecker product with qubit n-1 leftmost; bit q of (x, z) picks the factor."""
    m = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        f = {(0, 0): I2, (1, 0): X2, (0, 1): Z2, (1, 1): Y2}[(xb, zb)]
        m = np.kron(m, f)
    return m


def pauli_sum_dense(n: int, xs, zs, cs) -> np.ndarray:
    m = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for x, z, c in zip(xs, zs, cs):
        m += c * pauli_string_dense(n, int(x), int(z))
    return m


def jw_annihilator(n: int, j: int) -> sp.csr_matrix:
    """a_j |occ> = (-1)^{#occupied modes below j} |occ without j>, 0 if j empty."""
    dim = 1 << n
    rows, cols, vals = [], [], []
    for occ in range(dim):
        if (occ >> j) & 1:
            sign = -1.0 if bin(occ & ((1 << j) - 1)).count("1") % 2 else 1.0
            rows.append(occ ^ (1 << j))
            cols.append(occ)
            vals.append(sign)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim), dtype=np.complex128)


def encoding_permutation(beta: np.ndarray) -> sp.csr_matrix:
    """P_beta |occ> = |beta occ mod 2>."""
    n = beta.shape[0]
    dim = 1 << n
    b = np.zeros(dim, dtype=np.int64)
    for occ in range(dim):
        v = np.array([(occ >> k) & 1 for k in range(n)])
        bits = (beta.astype(np.int64) @ v) & 1
        b[occ] = int(sum(int(bit) << q for q, bit in enumerate(bits)))
    return sp.csr_matrix((np.ones(dim), (b, np.arange(dim))), shape=(dim, dim), dtype=np.complex128)


def annihilators(n: int, beta: np.ndarray | None = None) -> list:
    a = [jw_annihilator(n, j) for j in range(n)]
    if beta is None:
        return a
    p = encoding_permutation(beta)
    return [(p @ aj @ p.T).tocsr() for aj in a]


def fermion_hamiltonian(h: np.ndarray, g: np.ndarray, e_const: float,
                        beta: np.ndarray | None = None) -> sp.csr_matrix:
    """Eq. 2 with h_ijkl = (p_i p_k | p_j p_l) for matching spins; m = 2p + spin."""
    n_orb = h.shape[0]
    n = 2 * n_orb
    a = annihilators(n, beta)
    ad = [x.conj().T.tocsr() for x in a]
    dim = 1 << n
    H = sp.identity(dim, dtype=np.complex128, format="csr") * e_const
    spin = [m % 2 for m in range(n)]
    orb = [m // 2 for m in range(n)]
    for i in range(n):
        for j in range(n):
            if spin[i] == spin[j] and h[orb[i], orb[j]] != 0.0:
                H = H + h[orb[i], orb[j]] * (ad[i] @ a[j])
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            adij = ad[i] @ ad[j]
            for k in range(n):
                if spin[k] != spin[i]:
                    continue
                for l in range(n):
                    if l == k or spin[l] != spin[j]:
                        continue
                    v = g[orb[i], orb[k], orb[j], orb[l]]
                    if v != 0.0:
                        H = H + (0.5 * v) * (adij @ a[l] @ a[k])
    return H.tocsr()


def excitation_generator(n: int, occ, vir, beta: np.ndarray | None = None) -> sp.csr_matrix:
    """A = T - T^+ with T = a_a^+ a_i or a_a^+ a_b^+ a_j a_i."""
    a = annihilators(n, beta)
    if len(occ) == 1:
        T = a[vir[0]].conj().T @ a[occ[0]]
    else:
        i, j = occ
        aa, bb = vir
        T = a[aa].conj().T @ a[bb].conj().T @ a[j] @ a[i]
    return (T - T.conj().T).tocsr()


def expm_antihermitian(theta: float, A: np.ndarray) -> np.ndarray:
    """exp(theta A) for anti-Hermitian A through eigh of the Hermitian iA."""
    w, v = np.linalg.eigh(1j * A)
    # A = -i (iA) = -i V diag(w) V^+
    return (v * np.exp(-1j * theta * w)) @ v.conj().T


def taylor5_dense(theta: float, A: np.ndarray) -> np.ndarray:
    """sum_{k=0..5} (theta A)^k / k! as a dense matrix (Eq. 6)."""
    out = np.eye(A.shape[0], dtype=np.complex128)
    term = np.eye(A.shape[0], dtype=np.complex128)
    for k in range(1, 6):
        term = term @ (theta * A) / k
        out = out + term
    return out


def sector_mask(n: int, n_alpha: int, n_beta: int, beta: np.ndarray | None = None) -> np.ndarray:
    """Boolean mask over qubit basis states of the (n_alpha, n_beta) sector."""
    dim = 1 << n
    occ = np.arange(dim)
    na = sum(((occ >> m) & 1) for m in range(0, n, 2))
    nb = sum(((occ >> m) & 1) for m in range(1, n, 2))
    mask = (na == n_alpha) & (nb == n_beta)
    if beta is None:
        return mask
    p = encoding_permutation(beta)
    return (p @ mask.astype(np.complex128)).real > 0.5


def fidelity(a: np.ndarray, b: np.ndarray) -> float:
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))
