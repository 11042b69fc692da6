"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle (oracle.c, built with gcc and both sanitizers) runs a whole
  adaptive step on an 8-qubit workload: CSR build (with a refused bad mask),
  energy, gradients, selection, Taylor-5, renormalisation, one more product.
  Its results are bit-identical to the regular build's.
* libadaptvqe's host-only entry points (the library's sources built by hipcc
  with the sanitizers on the host side only; device code is compiled as usual
  and never launched): vqe_mf_describe, vqe_mf_pool_create / get / owner_rows
  / destroy on the JW and BK pools at 8 qubits, vqe_partition_greedy on a
  seeded random graph, and their refusals of bad arguments.  Results equal the
  regular library's, called through the binding.

A sanitizer report, a leak or a non-zero exit fails the test.  The builds are
cached under _build/sanitize/, keyed by a hash of their sources.
"""
import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_29692_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
CACHE = os.path.join(ROOT, "_build", "sanitize")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:exitcode=23",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=24",
           "OMP_NUM_THREADS": "4"}


def _hash(paths, extra=""):
    h = hashlib.sha256(extra.encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)} failed ({r.returncode}):\n{r.stdout[-2000:]}\n"
                           f"{r.stderr[-4000:]}")
    return r


def _sanitized(stdout_stderr: str):
    for marker in ("AddressSanitizer", "LeakSanitizer", "runtime error:", "UndefinedBehavior"):
        assert marker not in stdout_stderr, stdout_stderr[-4000:]


@pytest.fixture(scope="module")
def oracle_exe():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    srcs = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c")]
    out_dir = os.path.join(CACHE, "oracle-" + _hash(srcs))
    exe = os.path.join(out_dir, "oracle_driver")
    if not os.path.exists(exe):
        os.makedirs(out_dir, exist_ok=True)
        _run(["gcc", "-O2", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-o", exe + ".tmp", *srcs, "-lm"])
        os.replace(exe + ".tmp", exe)
    return exe


@pytest.fixture(scope="module")
def abi_exe():
    from paper_2606_29692_amd import build as PBUILD
    try:
        hipcc = PBUILD.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    names = list(PBUILD.SOURCES)
    srcs = [os.path.join(CSRC, n) for n in names]
    hdrs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp"))
    drv = os.path.join(HERE, "host_abi_driver.cpp")
    inc = os.path.join(ROOT, "include", "adaptvqe.h")
    out_dir = os.path.join(CACHE, "abi-" + _hash(srcs + hdrs + [drv, inc]))
    exe = os.path.join(out_dir, "host_abi_driver")
    if not os.path.exists(exe):
        os.makedirs(out_dir, exist_ok=True)
        san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
        flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *san]

        def comp(src):
            obj = os.path.join(out_dir, os.path.basename(src) + ".o")
            _run([hipcc, *flags, "-c", src, "-o", obj])
            return obj

        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(comp, srcs + [drv]))
        _run([hipcc, "--offload-arch=gfx950", "-g", *san, "-o", exe + ".tmp", *objs])
        os.replace(exe + ".tmp", exe)
    return exe


def _pack_lines(pack, tol=None):
    c = np.asarray(pack.coeff, dtype=np.complex128)
    lines = [f"{len(c)}" + (f" {float(tol)!r}" if tol is not None else "")]
    for x, z, v in zip(pack.xmask, pack.zmask, c):
        lines.append(f"{int(x)} {int(z)} {float(v.real)!r} {float(v.imag)!r}")
    return lines


def test_oracle_under_sanitizers(oracle_exe):
    s = vs.make_system(vs.SystemSpec(8, 4, "jw", False, vs.system_seed(91, 0), e_const=0.25))
    psi = vs.complex_start_state(s)
    theta = 0.07
    lines = ["8"] + _pack_lines(s.hamiltonian, orc.default_tol(s.hamiltonian.coeff))
    lines.append(str(len(s.pool)))
    for p in s.pool:
        lines += _pack_lines(p, orc.default_tol(p.coeff))
    lines += [f"{float(v.real)!r} {float(v.imag)!r}" for v in psi]
    lines.append(repr(theta))
    r = subprocess.run([oracle_exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env={**os.environ, **SAN_ENV}, timeout=300)
    _sanitized(r.stdout + r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    out = {}
    psi_d, hpsi_d, g_d = [], [], []
    for ln in r.stdout.splitlines():
        f = ln.split()
        if f[0] == "psi":
            psi_d.append(complex(float(f[1]), float(f[2])))
        elif f[0] == "hpsi":
            hpsi_d.append(complex(float(f[1]), float(f[2])))
        elif f[0] == "g":
            g_d.append(float(f[2]))
        else:
            out[f[0]] = f[1:]
    # the regular build, through the Python front end
    oH = orc.csr_from_pack(s.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in s.pool]
    e, n2, im, sigma = orc.energy(oH, psi)
    g = orc.gradients(pool, psi, sigma)
    k, gmax = orc.select(g)
    nxt, nn = orc.normalize(orc.taylor5(pool[k], theta, psi))
    assert int(out["nnz"][0]) == oH.nnz
    assert [float(v) for v in out["energy"]] == [e, n2, im]
    assert g_d == list(g)
    assert int(out["select"][0]) == k and float(out["select"][1]) == gmax
    assert float(out["norm2"][0]) == nn
    assert np.array_equal(np.array(psi_d), nxt)
    assert np.array_equal(np.array(hpsi_d), orc.spmv(oH, nxt))


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_host_abi_under_sanitizers(abi_exe, mapping):
    from paper_2606_29692_amd import binding as B
    s = vs.make_system(vs.SystemSpec(8, 4, mapping, False, 3))
    M = len(s.pool)
    rng = np.random.default_rng(np.random.SeedSequence([92, 0]))
    K = 40
    a = rng.random((K, K)) < 0.3
    adj = np.triu(a, 1)
    adj = (adj | adj.T).astype(np.uint8)
    lines = [f"8 {M}"]
    for p in s.pool:
        lines += _pack_lines(p)
    lines.append(str(K))
    lines += [" ".join(str(int(v)) for v in row) for row in adj]
    r = subprocess.run([abi_exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env={**os.environ, **SAN_ENV}, timeout=300)
    _sanitized(r.stdout + r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    got = r.stdout.splitlines()
    # the regular library through the binding (host calls only)
    mfp = B.MfPool(s.pool)
    try:
        exp = []
        for j, p in enumerate(s.pool):
            d = B.mf_describe(p, 1e-12)
            exp.append(_desc_line("describe", j, d))
        exp.append("pool_create rc 0")
        for j in range(M):
            exp.append(_desc_line("get", j, mfp.get(j)))
            for tile in (-1, 0, 1):
                rows, idx = mfp.owner_rows(j, 128, tile)
                exp.append(f"owner {j} {tile} {len(rows)}" +
                           "".join(f" {int(a)}:{int(b)}" for a, b in zip(rows, idx)))
    finally:
        mfp.close()
    fam = B.partition_greedy(adj)
    exp.append(f"families {int(fam.max()) + 1}" + "".join(f" {int(v)}" for v in fam))
    assert got[:len(exp)] == exp
    assert len(got) == len(exp) + 6


def _desc_line(tag, j, d):
    s = (f"{tag} {j} rc 0 x {d['x']} zsign {d['zsign']} v {_g17(d['v'].real)} "
         f"{_g17(d['v'].imag)} ncon {len(d['beta'])} kbits {d['kbits']}")
    return s + "".join(f" {b}" for b in d["beta"])


def _g17(v: float) -> str:
    return f"{v:.17g}"
