"""Seeded synthetic inputs for the adaptive-VQE hot path.

This package produces the inputs both the HIP path and the CPU oracle consume:
molecule-shaped random integrals, the second-quantised Hamiltonian (Eq. 2)
mapped to a Pauli sum (Eq. 3) under Jordan-Wigner or Bravyi-Kitaev (Sec. II-A),
the excitation pool (Sec. III-E) as Pauli packs, the reference determinant and
the rotation angles.  It performs none of the method's own arithmetic (no CSR
compilation, no sparse products, no Taylor update, energy or gradient).
"""
from .configs import (ELECTRONS, System, SystemSpec, complex_start_state, config_c1, config_c2,
                      config_c3, config_c4, config_c5, make_system, reference_state,
                      sector_indices, shared_pool, system_seed)
from .encoding import bk_matrix, encode_bits, encoding_matrix, gf2_inverse, jw_matrix, ladder_table
from .fermion import (Excitation, PauliPack, excitation_list, generator_pack, hamiltonian_pack,
                      pool_packs, pool_size_formula, reference_occupation)
from .integrals import Integrals, draw_thetas, gen_integrals, rng_for
from .pauli import from_labels, merge, multiply, popcount, to_labels
