"""The C ABI from plain C: the header is valid ISO C11, and a C program
(tests/c_api_demo.c) that builds a Hamiltonian and a generator from Pauli
terms, takes the energy, applies the fifth-order update and takes the energy
again links against the library (CPU) and reproduces the oracle (GPU, 1e-12).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2606_29692_amd")
ROCM_INC = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"

needs_gcc = pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir(ROCM_INC),
                               reason="gcc or the ROCm headers are not available")


def compile_demo(out_dir) -> str:
    exe = os.path.join(str(out_dir), "c_api_demo")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           "-I", ROCM_INC, "-D__HIP_PLATFORM_AMD__", os.path.join(ROOT, "tests", "c_api_demo.c"),
           "-L", PKG, "-ladaptvqe", f"-Wl,-rpath,{PKG}", "-L", ROCM_LIB, "-lamdhip64",
           f"-Wl,-rpath,{ROCM_LIB}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@needs_gcc
def test_header_is_iso_c11():
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-fsyntax-only", "-x", "c", os.path.join(ROOT, "include", "adaptvqe.h")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@needs_gcc
def test_c_program_compiles_and_links(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libadaptvqe.so")):
        pytest.skip("libadaptvqe.so is not built")
    assert os.path.exists(compile_demo(tmp_path))


def oracle_energies():
    """The same operators as the C program, through the oracle."""
    n = 4
    H = vs.PauliPack(n, np.array([0, 0, 0, 0, 3, 3, 0, 12], dtype=np.uint64),
                     np.array([1, 2, 4, 8, 0, 3, 3, 0], dtype=np.uint64),
                     np.array([0.5, 0.3, -0.2, 0.1, 0.25, 0.25, 0.15, 0.05], dtype=np.complex128))
    A = vs.PauliPack(n, np.array([3], dtype=np.uint64), np.array([2], dtype=np.uint64),
                     np.array([1j], dtype=np.complex128))
    h, a = orc.csr_from_pack(H), orc.csr_from_pack(A)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[1] = 1.0
    e0 = orc.energy(h, psi)[0]
    phi, _ = orc.normalize(orc.taylor5(a, 0.3, psi))
    return e0, orc.energy(h, phi)[0]


def test_oracle_side_of_the_c_program():
    # on |0001> only the Z terms act diagonally: Z0 -> -1, Z1, Z2, Z3 -> +1,
    # Z0 Z1 -> -1; the update moves the state, so the energy changes
    e0, e1 = oracle_energies()
    assert abs(e0 - (-0.5 + 0.3 - 0.2 + 0.1 - 0.15)) < 1e-15
    assert abs(e1 - e0) > 1e-3


@needs_gcc
@pytest.mark.gpu
def test_c_program_matches_oracle(tmp_path):
    exe = compile_demo(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    vals = dict(line.split() for line in r.stdout.strip().splitlines())
    e0, e1 = oracle_energies()
    print(f"C program: E0 {vals['E0']} E1 {vals['E1']}; oracle {e0:.17g} {e1:.17g}")
    assert abs(float(vals["E0"]) - e0) <= 1e-12
    assert abs(float(vals["E1"]) - e1) <= 1e-12
