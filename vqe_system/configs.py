"""Workload definitions (synthetic stand-ins for the paper's molecules).

The paper runs H2O (12 qubits, pool 92) and BeH2 (14 qubits, pool 204) active
spaces (Table II).  Their integrals are not available; every system here is a
seeded synthetic one of the same shape (qubits, electrons, pool, 2^N).

Electron counts per register size: {8: 4, 10: 4, 12: 8, 14: 6, 16: 8}.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .encoding import encode_bits, encoding_matrix
from .fermion import (PauliPack, excitation_list, hamiltonian_pack, pool_packs,
                      reference_occupation)
from .integrals import STREAM_START, Integrals, draw_thetas, gen_integrals, rng_for

ELECTRONS = {4: 2, 6: 2, 8: 4, 10: 4, 12: 8, 14: 6, 16: 8, 18: 8, 20: 10}


def system_seed(cfg_id: int, state: int) -> int:
    """One integer seed per (workload, state) pair."""
    return int(np.random.SeedSequence([int(cfg_id), int(state)]).generate_state(1)[0])


@dataclass(frozen=True)
class SystemSpec:
    n_qubits: int
    n_electrons: int
    mapping: str = "jw"
    stretched: bool = False
    seed: int = 0
    e_const: float = 0.0


@dataclass
class System:
    spec: SystemSpec
    integrals: Integrals
    hamiltonian: PauliPack
    pool: list = field(default_factory=list)   # list[PauliPack]
    reference_index: int = 0                   # qubit basis index of the reference state

    @property
    def dim(self) -> int:
        return 1 << self.spec.n_qubits


_POOL_CACHE: dict = {}


def shared_pool(n_qubits: int, n_electrons: int, mapping: str) -> list:
    """Pool packs do not depend on the integrals; build each (N, n_e, mapping) once."""
    key = (n_qubits, n_electrons, mapping)
    if key not in _POOL_CACHE:
        _POOL_CACHE[key] = pool_packs(n_qubits, n_electrons, mapping)
    return _POOL_CACHE[key]


def make_system(spec: SystemSpec, with_pool: bool = True) -> System:
    ints = gen_integrals(spec.n_qubits // 2, spec.seed, spec.stretched, spec.e_const)
    ham = hamiltonian_pack(ints, spec.mapping)
    pool = shared_pool(spec.n_qubits, spec.n_electrons, spec.mapping) if with_pool else []
    beta = encoding_matrix(spec.mapping, spec.n_qubits)
    ref = encode_bits(beta, reference_occupation(spec.n_electrons))
    return System(spec, ints, ham, pool, ref)


def reference_state(sys: System, dtype=np.complex128) -> np.ndarray:
    psi = np.zeros(sys.dim, dtype=dtype)
    psi[sys.reference_index] = 1.0
    return psi


def sector_indices(sys: System) -> np.ndarray:
    """Qubit basis indices of every determinant with the reference's numbers of
    alpha (even spin-orbitals) and beta (odd) electrons, encoded by the
    system's mapping; ascending."""
    n = sys.spec.n_qubits
    occ = np.arange(1 << n, dtype=np.int64)
    ref = reference_occupation(sys.spec.n_electrons)

    def count(v, parity):
        return sum(((v >> m) & 1) for m in range(parity, n, 2))

    keep = (count(occ, 0) == count(ref, 0)) & (count(occ, 1) == count(ref, 1))
    dets = occ[keep]
    if sys.spec.mapping == "jw":
        return dets
    beta = encoding_matrix(sys.spec.mapping, n)
    return np.sort(np.array([encode_bits(beta, int(d)) for d in dets], dtype=np.int64))


def complex_start_state(sys: System, eps: float = 0.1, dtype=np.complex128) -> np.ndarray:
    """A seeded complex start state in the reference's particle sector: the
    reference determinant plus eps times a complex Gaussian vector over the
    sector (unit expected norm), scaled to unit norm.  Every amplitude outside
    the sector is exactly zero, and almost every amplitude inside it has a
    non-zero imaginary part, so products with it run in complex arithmetic."""
    idx = sector_indices(sys)
    rng = rng_for(sys.spec.seed, STREAM_START)
    z = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
    psi = np.zeros(sys.dim, dtype=np.complex128)
    psi[idx] = eps * z / np.sqrt(2.0 * idx.size)
    psi[sys.reference_index] += 1.0
    psi /= np.linalg.norm(psi)
    return psi.astype(dtype)


# The five workloads.  Each returns a list of SystemSpec and a theta seed.
def config_c1():
    """N=8 (4 orbitals, 4 electrons), JW, 5 adaptive steps."""
    return [SystemSpec(8, 4, "jw", False, system_seed(1, 0))], 5


def config_c2():
    """N=12 (6 orbitals, 8 electrons), JW and BK, equilibrium and stretched, 20 steps."""
    specs = [SystemSpec(12, 8, m, st, system_seed(2, 0)) for m in ("jw", "bk") for st in (False, True)]
    return specs, 20


def config_c3():
    """N=14 (7 orbitals, 6 electrons), JW, 30 steps."""
    return [SystemSpec(14, 6, "jw", False, system_seed(3, 0))], 30


def config_c4(n_states: int = 64, mixed: bool = True):
    """Batched launch: n_states independent states, N cycling over (10, 12, 14)
    when mixed, else all at N=14; one update per state per step."""
    specs = []
    for s in range(n_states):
        n = (10, 12, 14)[s % 3] if mixed else 14
        specs.append(SystemSpec(n, ELECTRONS[n], "jw", False, system_seed(4 if mixed else 44, s)))
    return specs, 1


def config_c5(n_runs: int = 64, sizes=(8, 10, 12, 14, 16), seed: int = 5):
    """Serving: resident runs with N drawn uniformly from ``sizes``."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    ns = rng.choice(np.asarray(sizes), size=n_runs)
    return [SystemSpec(int(n), ELECTRONS[int(n)], "jw", False, system_seed(5, r))
            for r, n in enumerate(ns)], 1


__all__ = ["SystemSpec", "System", "make_system", "reference_state", "shared_pool",
           "sector_indices", "complex_start_state",
           "system_seed", "draw_thetas", "excitation_list", "ELECTRONS",
           "config_c1", "config_c2", "config_c3", "config_c4", "config_c5"]
