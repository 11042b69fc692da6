"""Fermion-to-qubit encodings: Jordan-Wigner and Bravyi-Kitaev (Sec. II-A).

Both are linear encodings over GF(2): a fermionic occupation vector n (bit m =
occupation of spin-orbital m) is stored in the qubit register as b = beta n
(mod 2).

* Jordan-Wigner (Eq. 4): beta = I.  The ladder operator a_m carries a Z string
  on the lower modes, i.e. the sign (-1)^{popcount(n & ((1<<m)-1))}.  The paper
  writes the Z string on the modes after j in Kronecker order; with mode j kept
  in bit N-j that is the same parity-of-lower-modes rule, which is the
  convention used here.
* Bravyi-Kitaev (binary-tree parity/occupation encoding, Sec. II-A): the paper
  gives no formula.  The Fenwick-tree form is used: qubit i stores the parity of
  modes k with (i & (i+1)) <= k <= i.  For N a power of two this is the
  Seeley-Richard-Love matrix; for other N it is its leading N x N block.

For any invertible beta the annihilator acts on a qubit basis state |b> as

    a_j |b> = [n_j = 1] (-1)^{sum_{k<j} n_k} |b ^ u_j>,

with n = beta^{-1} b and u_j = column j of beta.  With w_j = row j of beta^{-1}
and p_j = XOR of rows k < j of beta^{-1} this is the Pauli sum

    a_j = 1/2 X^{u_j} Z^{p_j} - 1/2 X^{u_j} Z^{p_j ^ w_j},

and a_j^dagger has the complex-conjugate coefficients on the same strings
(every P(x, z) is Hermitian).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .pauli import xz_word_to_p

MAPPINGS = ("jw", "bk")


def jw_matrix(n: int) -> np.ndarray:
    return np.eye(n, dtype=np.uint8)


def bk_matrix(n: int) -> np.ndarray:
    beta = np.zeros((n, n), dtype=np.uint8)
    for i in range(n):
        lo = i & (i + 1)
        beta[i, lo:i + 1] = 1
    return beta


def encoding_matrix(mapping: str, n: int) -> np.ndarray:
    if mapping == "jw":
        return jw_matrix(n)
    if mapping == "bk":
        return bk_matrix(n)
    raise ValueError(f"unknown mapping {mapping!r}; expected one of {MAPPINGS}")


def gf2_inverse(a: np.ndarray) -> np.ndarray:
    """Inverse of a square 0/1 matrix over GF(2) (Gauss-Jordan)."""
    n = a.shape[0]
    m = np.concatenate([a.astype(np.uint8) & 1, np.eye(n, dtype=np.uint8)], axis=1)
    for col in range(n):
        piv = next((r for r in range(col, n) if m[r, col]), None)
        if piv is None:
            raise ValueError("matrix is singular over GF(2)")
        if piv != col:
            m[[col, piv]] = m[[piv, col]]
        for r in range(n):
            if r != col and m[r, col]:
                m[r] ^= m[col]
    return m[:, n:]


def _rowmask(row) -> int:
    return int(sum(1 << q for q, v in enumerate(row) if v))


def encode_bits(beta: np.ndarray, n_occ: int) -> int:
    """b = beta n (mod 2) for an occupation bit mask n."""
    nvec = np.array([(n_occ >> k) & 1 for k in range(beta.shape[0])], dtype=np.int64)
    b = (beta.astype(np.int64) @ nvec) & 1
    return _rowmask(b)


@lru_cache(maxsize=None)
def ladder_table(mapping: str, n: int):
    """Pauli expansion of every annihilator a_j, j = 0..n-1.

    Returns (x, z, c) arrays of shape (n, 2): a_j = sum_s c[j,s] P(x[j,s], z[j,s]).
    The creator a_j^dagger is sum_s conj(c[j,s]) P(x[j,s], z[j,s]).
    """
    beta = encoding_matrix(mapping, n)
    binv = gf2_inverse(beta)
    x = np.zeros((n, 2), dtype=np.uint64)
    z = np.zeros((n, 2), dtype=np.uint64)
    c = np.zeros((n, 2), dtype=np.complex128)
    p = 0
    for j in range(n):
        u = _rowmask(beta[:, j])
        w = _rowmask(binv[j, :])
        x[j, :] = u
        z[j, 0] = p
        z[j, 1] = p ^ w
        c[j, 0] = xz_word_to_p(u, p, 0.5)
        c[j, 1] = xz_word_to_p(u, p ^ w, -0.5)
        p ^= w
    x.setflags(write=False)
    z.setflags(write=False)
    c.setflags(write=False)
    return x, z, c
