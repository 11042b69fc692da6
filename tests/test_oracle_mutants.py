"""Planted mistakes in the oracle must be caught by the pins.

Each mutant is a copy of oracle.c with one plausible slip (a dropped term, a
wrong sign or index, a missing conjugate, a wrong factor), compiled on the
CPU into a temporary library.  A compact version of the pins runs against it
and must report at least one failure; against the real oracle it must report
none.
"""
import contextlib
import os
import subprocess
import tempfile

import numpy as np
import pytest

import dense_ref as D
import vqe_system as vs
from oracle import oracle as orc

MUTANTS = {
    "taylor_no_factorial": ("c = c * theta / (double)n;", "c = c * theta;"),
    "taylor_order_four": ("for (int n = 1; n <= 5; n++)", "for (int n = 1; n <= 4; n++)"),
    "taylor_skips_psi": ("memcpy(acc, psi, 2 * (size_t)dim * sizeof(double));",
                         "memset(acc, 0, 2 * (size_t)dim * sizeof(double));"),
    "phase_i_sign": ("case 1: re = -cim; im = cre;  break;", "case 1: re = cim; im = -cre;  break;"),
    "z_sign_on_row": ("if (popcount64(z & col) & 1)", "if (popcount64(z & (col ^ x)) & 1)"),
    "drop_rule_or": ("if (fabs(re) <= tol && fabs(im) <= tol)",
                     "if (fabs(re) <= tol || fabs(im) <= tol)"),
    "spmv_row_index": ("double c = x[2 * col[k]], d = x[2 * col[k] + 1];",
                       "double c = x[2 * r], d = x[2 * r + 1];"),
    "spmv_cross_sign": ("im = im + (a * d + b * c);", "im = im + (a * d - b * c);"),
    "energy_no_conj": ("nre = nre + (a * c + b * d);", "nre = nre + (a * c - b * d);"),
    "gradient_no_two": ("g[j] = 2.0 * s;", "g[j] = s;"),
    "gradient_imag_part": ("s = s + (sigma[2 * r] * work[2 * r] + sigma[2 * r + 1] * work[2 * r + 1]);",
                           "s = s + (sigma[2 * r] * work[2 * r + 1] - sigma[2 * r + 1] * work[2 * r]);"),
    "select_signed": ("if (fabs(g[j]) > gmax)", "if (g[j] > gmax)"),
    "select_last_tie": ("for (int32_t j = 0; j < M; j++)\n        if (fabs(g[j]) >= gmax * (1.0 - rel_tie))",
                        "for (int32_t j = M - 1; j >= 0; j--)\n        if (fabs(g[j]) >= gmax * (1.0 - rel_tie))"),
}


@contextlib.contextmanager
def _using_library(path):
    saved_lib, saved_path = orc._lib, orc.LIB_PATH
    orc._lib = None
    orc.LIB_PATH = path
    try:
        orc.lib()
        yield
    finally:
        orc._lib, orc.LIB_PATH = saved_lib, saved_path


def _pin_failures() -> list:
    """Small versions of the oracle pins; returns the names of those that fail."""
    fails = []
    rng = np.random.default_rng(123)
    # CSR of a random complex Pauli sum vs the Kronecker sum (P-1)
    n, T = 4, 25
    x = rng.integers(0, 16, T).astype(np.uint64)
    z = rng.integers(0, 16, T).astype(np.uint64)
    c = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    c[3] = 1e-3j                     # a term with a purely imaginary coefficient
    m = orc.csr_build(n, x, z, c)
    Pd = D.pauli_sum_dense(n, x, z, c)
    if not np.allclose(m.dense(), Pd, atol=1e-13):
        fails.append("csr")
    v = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    if not np.allclose(orc.spmv(m, v), Pd @ v, atol=1e-12):
        fails.append("spmv-complex")
    # system at N = 8
    s = vs.make_system(vs.SystemSpec(8, 4, "jw", False, 77))
    H = orc.csr_from_pack(s.hamiltonian)
    Hd = D.fermion_hamiltonian(s.integrals.h, s.integrals.g, 0.0).toarray()
    psi = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    if not np.allclose(orc.spmv(H, psi), Hd @ psi, atol=1e-12):
        fails.append("spmv")
    e, _, _, sigma = orc.energy(H, psi)
    if abs(e - (np.vdot(psi, Hd @ psi) / np.vdot(psi, psi)).real) > 1e-12:
        fails.append("energy")
    exc = vs.excitation_list(8, 4)
    pool = [orc.csr_from_pack(p) for p in s.pool]
    g = orc.gradients(pool, psi, Hd @ psi)
    for j in (0, 10, 25):
        Ad = D.excitation_generator(8, exc[j].occ, exc[j].vir).toarray()
        if abs(g[j] - np.vdot(psi, (Hd @ Ad - Ad @ Hd) @ psi).real) > 1e-11:
            fails.append("gradient")
            break
    Ad = D.excitation_generator(8, exc[5].occ, exc[5].vir).toarray()
    if not np.allclose(orc.taylor5(pool[5], 0.3, psi), D.taylor5_dense(0.3, Ad) @ psi, atol=1e-12):
        fails.append("taylor")
    if (orc.select([0.2, -0.9, 0.9, 0.1])[0] != 1 or orc.select([0.2, 0.9, -0.3])[0] != 1
            or orc.select([0.5, -0.9]) != (1, 0.9)):
        fails.append("select")
    return fails


def test_real_oracle_passes_compact_pins():
    assert _pin_failures() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    with open(orc.SRC_PATH) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "mutant.c")
        lpath = os.path.join(d, "libmutant.so")
        with open(cpath, "w") as f:
            f.write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fopenmp", "-o", lpath, cpath, "-lm"], check=True)
        with _using_library(lpath):
            fails = _pin_failures()
    assert fails, f"mutant {name} was not caught by any pin"
