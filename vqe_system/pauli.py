"""Pauli strings in (x, z) bit-mask form and their products.

A Pauli string on N qubits is stored as two bit masks: bit q of ``x`` and of
``z`` give the single-qubit factor on qubit q, with (0,0)=I, (1,0)=X, (0,1)=Z
and (1,1)=Y.  Because Y = i X Z, the string with masks (x, z) equals

    P(x, z) = i^{popcount(x & z)} X^x Z^z,

and it acts on a computational basis state |c> (bit q of c = qubit q) as

    P(x, z) |c> = i^{popcount(x & z)} (-1)^{popcount(z & c)} |c ^ x>.

This is the qubit form of a Pauli-sum operator (Sec. II-A, Eq. 3).  The
module only holds the algebra needed to *generate* inputs (fermion-to-qubit
mappings, excitation generators); it does no CSR compilation, no SpMV and no
state update.
"""
from __future__ import annotations

import numpy as np

# i^k for k = 0..3
IPOW = np.array([1.0 + 0.0j, 1.0j, -1.0 + 0.0j, -1.0j], dtype=np.complex128)


def popcount(a) -> np.ndarray:
    """Number of set bits of each element (as int64)."""
    return np.bitwise_count(np.asarray(a, dtype=np.uint64)).astype(np.int64)


def xz_word_to_p(x, z, coeff):
    """Rewrite ``coeff * X^x Z^z`` as ``coeff' * P(x, z)``.

    From P(x, z) = i^{|x&z|} X^x Z^z it follows that X^x Z^z = (-i)^{|x&z|} P(x, z).
    """
    k = popcount(np.asarray(x, dtype=np.uint64) & np.asarray(z, dtype=np.uint64)) % 4
    return np.asarray(coeff, dtype=np.complex128) * IPOW[(4 - k) % 4]


def multiply(x1, z1, c1, x2, z2, c2):
    """Product (c1 P(x1,z1)) (c2 P(x2,z2)) = c3 P(x1^x2, z1^z2), element-wise.

    Writing P = i^a X^x Z^z and moving Z^{z1} past X^{x2} (ZX = -XZ on every
    qubit where both act) gives the phase i^{a1 + a2 - a3 + 2|z1 & x2|}.
    """
    x1 = np.asarray(x1, dtype=np.uint64)
    z1 = np.asarray(z1, dtype=np.uint64)
    x2 = np.asarray(x2, dtype=np.uint64)
    z2 = np.asarray(z2, dtype=np.uint64)
    x3 = x1 ^ x2
    z3 = z1 ^ z2
    e = popcount(x1 & z1) + popcount(x2 & z2) - popcount(x3 & z3) + 2 * popcount(z1 & x2)
    return x3, z3, np.asarray(c1) * np.asarray(c2) * IPOW[e % 4]


def merge(x, z, c, drop_below: float = 0.0):
    """Sum coefficients of equal (x, z) strings; drop terms with |c| <= drop_below.

    Returns the merged strings sorted by (x, z).
    """
    x = np.asarray(x, dtype=np.uint64).ravel()
    z = np.asarray(z, dtype=np.uint64).ravel()
    c = np.asarray(c, dtype=np.complex128).ravel()
    key = (x << np.uint64(32)) | z
    uk, inv = np.unique(key, return_inverse=True)
    re = np.bincount(inv, weights=c.real, minlength=uk.size)
    im = np.bincount(inv, weights=c.imag, minlength=uk.size)
    cm = re + 1j * im
    keep = np.abs(cm) > drop_below
    uk = uk[keep]
    return uk >> np.uint64(32), uk & np.uint64(0xFFFFFFFF), cm[keep]


_CHARS = np.array([b"I", b"X", b"Z", b"Y"])


def to_labels(n_qubits: int, x, z) -> np.ndarray:
    """Fixed-width character labels, one per string (the contiguous label
    buffer of the vectorized pool layout, Sec. III-E).  The leftmost character
    acts on qubit N-1 (Kronecker order), the rightmost on qubit 0."""
    x = np.asarray(x, dtype=np.uint64)
    z = np.asarray(z, dtype=np.uint64)
    out = np.empty((x.size, n_qubits), dtype="S1")
    for q in range(n_qubits):
        xb = ((x >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
        zb = ((z >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
        out[:, n_qubits - 1 - q] = _CHARS[xb + 2 * zb]
    return out.view(f"S{n_qubits}").ravel()


def from_labels(labels) -> tuple[int, np.ndarray, np.ndarray]:
    """Inverse of :func:`to_labels`: returns (n_qubits, x, z)."""
    labels = np.asarray(labels)
    n = labels.dtype.itemsize
    chars = labels.view("S1").reshape(-1, n)
    x = np.zeros(chars.shape[0], dtype=np.uint64)
    z = np.zeros(chars.shape[0], dtype=np.uint64)
    for pos in range(n):
        q = np.uint64(n - 1 - pos)
        col = chars[:, pos]
        xb = (col == b"X") | (col == b"Y")
        zb = (col == b"Z") | (col == b"Y")
        bad = ~((col == b"I") | xb | zb)
        if bad.any():
            raise ValueError("Pauli labels may only contain I, X, Y, Z")
        x |= xb.astype(np.uint64) << q
        z |= zb.astype(np.uint64) << q
    return n, x, z
