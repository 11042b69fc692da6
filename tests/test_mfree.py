"""Matrix-free generator form (host logic, no GPU).

The descriptor derived from a generator's Pauli terms must represent exactly
the operator the oracle's CSR build makes of the same terms: same support,
same values bit for bit.  The owner-row enumeration that the device kernels
run (mirrored on the host by the library) must visit every pair of the
support exactly once, on the tile the screen stages for it.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc
from paper_2606_29692_amd import binding as B

CASES = [(4, 2, "jw"), (6, 2, "jw"), (6, 2, "bk"), (8, 4, "jw"), (8, 4, "bk"), (10, 4, "jw"),
         (10, 4, "bk")]


def parity(a):
    a = np.asarray(a, dtype=np.uint64)
    out = np.zeros(a.shape, dtype=np.uint64)
    for b in range(64):
        out ^= (a >> np.uint64(b)) & np.uint64(1)
    return out.astype(bool)


def implied_entries(d, n):
    """(rows, cols, values) of the operator a descriptor represents."""
    c = np.arange(1 << n, dtype=np.uint64)
    ok = np.ones(c.shape, dtype=bool)
    for i, b in enumerate(d["beta"]):
        ok &= parity(c & np.uint64(b)) == bool((d["kbits"] >> i) & 1)
    c = c[ok]
    sign = np.where(parity(c & np.uint64(d["zsign"])), -1.0, 1.0)
    return c ^ np.uint64(d["x"]), c, sign * d["v"]


def csr_entries(csr):
    rp = np.asarray(csr.rowptr, dtype=np.int64)
    rows = np.repeat(np.arange(len(rp) - 1, dtype=np.uint64), np.diff(rp))
    return rows, np.asarray(csr.col, dtype=np.uint64), np.asarray(csr.val, dtype=np.complex128)


def as_sorted(rows, cols, vals):
    o = np.lexsort((cols, rows))
    return rows[o], cols[o], vals[o]


@pytest.mark.parametrize("n,ne,mapping", CASES)
def test_descriptor_equals_oracle_csr(n, ne, mapping):
    s = vs.make_system(vs.SystemSpec(n, ne, mapping, False, vs.system_seed(3, n)))
    for j, pack in enumerate(s.pool):
        d = B.mf_describe(pack)
        assert d["n_qubits"] == n and len(d["beta"]) <= B.VQE_MF_MAX_CON
        ri, ci, vi = as_sorted(*implied_entries(d, n))
        ro, co, vo = as_sorted(*csr_entries(orc.csr_from_pack(pack)))
        np.testing.assert_array_equal(ri, ro, err_msg=f"generator {j}")
        np.testing.assert_array_equal(ci, co, err_msg=f"generator {j}")
        # bit-exact values (the same ordered FP64 sum up to an exact sign)
        np.testing.assert_array_equal(vi, vo, err_msg=f"generator {j}")


def test_jw_constraint_counts():
    """Under JW a single excitation has one support constraint and a double
    three (nnz 2^(N-1) and 2^(N-3), the pool CSR sizes)."""
    s = vs.make_system(vs.SystemSpec(8, 4, "jw", False, 5))
    counts = [len(B.mf_describe(p)["beta"]) for p in s.pool]
    assert counts.count(1) == 8 and counts.count(3) == 18 and len(counts) == 26


def pool_tile_bits(xs, n, kt):
    """The screen's tile bits of every generator (flip masks xs), as lists of
    bit positions: each generator's kt highest bits outside its mask (bit 0
    excluded), unless the greedy cover the library documents -- repeatedly
    the kt-subset of bits 1..n-1 (candidates in descending mask order; the
    first wins a tie) that the most remaining generators avoid -- needs fewer
    distinct sets."""
    own = []
    for x in xs:
        b = [p for p in range(n - 1, 0, -1) if not (x >> p) & 1][:kt]
        own.append(sorted(b))
    cand = [m << 1 for m in range((1 << (n - 1)) - 1, -1, -1) if bin(m).count("1") == kt]
    out = [None] * len(xs)
    left = list(range(len(xs)))
    while left:
        counts = [sum(1 for j in left if not (xs[j] & c)) for c in cand]
        best = max(range(len(cand)), key=lambda i: (counts[i], -i))
        assert counts[best] > 0
        c = cand[best]
        for j in left:
            if not (xs[j] & c):
                out[j] = [p for p in range(n) if (c >> p) & 1]
        left = [j for j in left if out[j] is None]
    distinct = lambda v: len({tuple(t) for t in v})  # noqa: E731
    return out if distinct(out) < distinct(own) else own


def compress(a, tb):
    for p in sorted(tb, reverse=True):
        a = ((a >> (p + 1)) << p) | (a & ((1 << p) - 1))
    return a


@pytest.mark.parametrize("n,ne,mapping", [(6, 2, "jw"), (8, 4, "jw"), (8, 4, "bk"), (10, 4, "bk")])
def test_owner_rows_cover_every_pair_once(n, ne, mapping):
    s = vs.make_system(vs.SystemSpec(n, ne, mapping, False, vs.system_seed(4, n)))
    pool = B.MfPool(s.pool)
    dim = 1 << n
    tbs = {kt: pool_tile_bits([pool.get(j)["x"] for j in range(pool.M)], n, kt) for kt in (1, 2)}
    for j in range(pool.M):
        d = pool.get(j)
        h = d["x"].bit_length() - 1
        rows_all, _, _ = implied_entries(d, n)
        expect = np.sort(rows_all[((rows_all >> np.uint64(h)) & np.uint64(1)) == 0])
        # whole state (the update)
        rows, _ = pool.owner_rows(j, dim, -1)
        np.testing.assert_array_equal(np.sort(rows.astype(np.uint64)), expect)
        # screen tiles of dim / 2^kt rows
        for kt in (1, 2):
            tile_rows = dim >> kt
            tb = tbs[kt][j]
            assert not (d["x"] & sum(1 << p for p in tb)) and 0 not in tb
            seen = []
            for v in range(1 << kt):
                rows, idx = pool.owner_rows(j, tile_rows, v)
                r = rows.astype(np.int64)
                # tile bits of every row equal the tile's value
                vb = 0
                for b, p in enumerate(sorted(tb)):
                    vb |= ((v >> b) & 1) << p
                tmask = sum(1 << p for p in tb)
                assert np.all((r & tmask) == vb)
                # LDS indices: the row's compressed index, unique, in range;
                # the partner lies in the same tile
                ci = np.array([compress(int(a), tb) for a in r], dtype=np.int64)
                np.testing.assert_array_equal(idx.astype(np.int64), ci)
                assert len(np.unique(ci)) == len(ci) and (ci.size == 0 or ci.max() < tile_rows)
                assert np.all(((r ^ d["x"]) & tmask) == vb)
                seen.append(r)
            allr = np.sort(np.concatenate(seen)).astype(np.uint64)
            np.testing.assert_array_equal(allr, expect)
    pool.close()


def _pack(n, terms):
    return vs.PauliPack(n, np.array([t[0] for t in terms], dtype=np.uint64),
                        np.array([t[1] for t in terms], dtype=np.uint64),
                        np.array([t[2] for t in terms], dtype=np.complex128))


def test_single_pauli_string():
    """One Pauli string: support everywhere, value c i^{|x&z|}."""
    n = 5
    p = _pack(n, [(0b00110, 0b01100, 0.25)])
    d = B.mf_describe(p)
    assert d["beta"] == [] and d["zsign"] == 0b01100
    assert d["v"] == 0.25 * 1j ** bin(0b00110 & 0b01100).count("1")
    ri, ci, vi = as_sorted(*implied_entries(d, n))
    ro, co, vo = as_sorted(*csr_entries(orc.csr_from_pack(p)))
    np.testing.assert_array_equal(ri, ro)
    np.testing.assert_array_equal(vi, vo)


@pytest.mark.parametrize("terms", [
    [(0b011, 0b001, 1.0), (0b101, 0b000, 1.0)],                 # two flip masks
    [(0, 0b011, 1.0)],                                         # diagonal (x = 0)
    [(0b011, 0b001, 1.0), (0b011, 0b100, 0.5)],                # two surviving patterns
    [(0b011, 0b001, 0.5), (0b011, 0b001, -0.5)],               # cancels to zero
    [(0b011, 0b000, 1.0), (0b011, 0b001, -1j)],                # support not closed under ^x
])
def test_rejected_forms(terms):
    with pytest.raises(B.VqeError) as e:
        B.mf_describe(_pack(3, terms))
    assert e.value.status == -5


def test_hamiltonian_is_rejected():
    s = vs.make_system(vs.SystemSpec(6, 2, "jw", False, 1))
    with pytest.raises(B.VqeError):
        B.mf_describe(s.hamiltonian)
