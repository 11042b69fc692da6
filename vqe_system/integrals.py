"""Seeded, synthetic, molecule-shaped electron integrals.

The paper's molecular integrals (H2O and BeH2 active spaces, Sec. IV) are not
available, so every Hamiltonian is built from random integrals with the same
shapes: n_orb spatial orbitals, a symmetric one-body matrix whose entries
decay away from the diagonal, and two-body integrals with the 8-fold
permutational symmetry of real chemist-notation integrals (pq|rs).

Recipe:
  * one-body:  h_pq ~ N(0, sigma_pq^2), sigma_pq = exp(-|p-q|), drawn on p <= q
    and mirrored; the diagonal is sorted ascending so that orbital index order
    is energy order (the aufbau reference fills the lowest indices);
  * stretched geometry variant: the diagonal gaps are shrunk five-fold,
    h_pp <- h_00 + (h_pp - h_00) / 5, which makes the reference nearly
    degenerate (strong correlation);
  * two-body:  (pq|rs) ~ N(0, 0.1^2) on canonical quadruples (p>=q, r>=s,
    pq>=rs) and copied to all 8 symmetric positions;
  * e_const: a scalar (identity) term, 0 unless asked for.

Random streams: numpy's default_rng seeded by SeedSequence([seed, stream]),
stream 0 for integrals, stream 1 for rotation angles, stream 4 for the
complex start states.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

STREAM_INTEGRALS = 0
STREAM_THETA = 1
STREAM_START = 4


def rng_for(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


@dataclass(frozen=True)
class Integrals:
    h: np.ndarray        # (n_orb, n_orb) symmetric
    g: np.ndarray        # (n_orb,)*4 chemist (pq|rs), 8-fold symmetric
    e_const: float

    @property
    def n_orb(self) -> int:
        return self.h.shape[0]


def gen_integrals(n_orb: int, seed: int, stretched: bool = False,
                  e_const: float = 0.0) -> Integrals:
    rng = rng_for(seed, STREAM_INTEGRALS)
    idx = np.arange(n_orb)
    sigma = np.exp(-np.abs(idx[:, None] - idx[None, :]).astype(np.float64))
    a = rng.standard_normal((n_orb, n_orb)) * sigma
    h = np.triu(a) + np.triu(a, 1).T
    d = np.sort(np.diag(h).copy())
    if stretched:
        d = d[0] + (d - d[0]) / 5.0
    h[idx, idx] = d

    g = np.zeros((n_orb,) * 4)
    for p in range(n_orb):
        for q in range(p + 1):
            pq = p * (p + 1) // 2 + q
            for r in range(n_orb):
                for s in range(r + 1):
                    rs = r * (r + 1) // 2 + s
                    if rs > pq:
                        continue
                    v = 0.1 * rng.standard_normal()
                    for (i, j, k, l) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                                         (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
                        g[i, j, k, l] = v
    return Integrals(h=h, g=g, e_const=float(e_const))


def draw_thetas(seed: int, count: int, lo: float = -0.1, hi: float = 0.1) -> np.ndarray:
    """Rotation angles for the adaptive loop, U(lo, hi) (a caller input; the
    paper describes no optimiser)."""
    return rng_for(seed, STREAM_THETA).uniform(lo, hi, size=count)
