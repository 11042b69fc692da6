"""ctypes front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does, and
this module imports nothing from the product package.

Every function follows a passage of the paper:
  csr_build  -- Pauli sum (Eq. 3) compiled to CSR (Sec. III-E)
  csr_rows, spmv_rows -- selected rows of that CSR and the product at them
                (sampled checks of operators too large to build whole)
  spmv       -- one sparse product (Eq. 7)
  taylor5    -- fifth-order update, Eq. 6 via Eq. 7 and Eq. 8
  normalize  -- unit-norm rescaling (the paper is silent; see the readings)
  energy     -- Rayleigh quotient (Eq. 1)
  gradients  -- pool gradients (Eq. 5) as 2 Re <H psi|A_j psi>
  select     -- argmax |g_j| with a stated tie rule (Sec. III-D)
  adapt_run  -- the adaptive loop of Sec. III-D with fixed step count
  step_energy, line_search -- the energy of the updated state as a function
                of the angle, and its minimiser (parameter optimisation, which
                Sec. III-D leaves implicit; see the readings)
  ansatz_state, ansatz_energy, reoptimize -- the state of the whole adaptive
                ansatz (every selected generator's update applied in order to
                the reference) and the cyclic coordinate minimisation of its
                energy over all angles (re-optimisation of the parameters)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

# Relative tolerance of the selection tie rule: candidates are all j with
# |g_j| >= max|g| * (1 - REL_TIE); the lowest index among them is chosen.
REL_TIE = 1e-6


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, OpenMP over rows)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, SRC_PATH, "-lm"],
                       check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_csr_build.restype = C.c_int64
        L.orc_csr_build.argtypes = [C.c_int, C.c_int64, _U64, _U64, _D, C.c_double, _I64,
                                    C.c_void_p, C.c_void_p]
        L.orc_csr_rows.restype = C.c_int64
        L.orc_csr_rows.argtypes = [C.c_int, C.c_int64, _U64, _U64, _D, C.c_double, _I64, C.c_int64,
                                   _I64, C.c_void_p, C.c_void_p]
        L.orc_spmv.restype = None
        L.orc_spmv.argtypes = [C.c_int64, _I64, _I32, _D, _D, _D]
        L.orc_taylor5.restype = None
        L.orc_taylor5.argtypes = [C.c_int64, _I64, _I32, _D, C.c_double, _D, _D, _D]
        L.orc_normalize.restype = C.c_double
        L.orc_normalize.argtypes = [C.c_int64, _D]
        L.orc_energy.restype = None
        L.orc_energy.argtypes = [C.c_int64, _I64, _I32, _D, _D, _D, _D]
        L.orc_gradients.restype = None
        L.orc_gradients.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    _D, _D, _D, _D]
        L.orc_select.restype = C.c_int32
        L.orc_select.argtypes = [C.c_int32, _D, C.c_double, C.POINTER(C.c_double)]
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_threads(int(n))


@dataclass
class CSR:
    n_qubits: int
    rowptr: np.ndarray   # int64[dim+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # complex128[nnz]

    @property
    def dim(self) -> int:
        return self.rowptr.size - 1

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        m = np.zeros((self.dim, self.dim), dtype=np.complex128)
        rows = np.repeat(np.arange(self.dim), np.diff(self.rowptr))
        m[rows, self.col] = self.val
        return m


def default_tol(coeff) -> float:
    """Drop threshold used by default: 1e-12 * max_t |c_t| (absolute)."""
    coeff = np.asarray(coeff)
    return 1e-12 * float(np.abs(coeff).max()) if coeff.size else 0.0


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def csr_build(n_qubits: int, xmask, zmask, coeff, tol: float | None = None) -> CSR:
    """CSR of sum_t coeff[t] P(xmask[t], zmask[t]) (see oracle.c, orc_csr_build)."""
    x = np.ascontiguousarray(xmask, dtype=np.uint64)
    z = np.ascontiguousarray(zmask, dtype=np.uint64)
    c = _c128(coeff)
    if tol is None:
        tol = default_tol(c)
    dim = 1 << n_qubits
    rowptr = np.zeros(dim + 1, dtype=np.int64)
    cd = c.view(np.float64)
    nnz = lib().orc_csr_build(n_qubits, x.size, x, z, cd, tol, rowptr, None, None)
    if nnz < 0:
        raise ValueError("oracle csr_build: bad arguments")
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    val = np.zeros(max(nnz, 1), dtype=np.complex128)
    lib().orc_csr_build(n_qubits, x.size, x, z, cd, tol, rowptr,
                        col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p))
    return CSR(n_qubits, rowptr, col[:nnz], val[:nnz])


def csr_from_pack(pack, tol: float | None = None) -> CSR:
    return csr_build(pack.n_qubits, pack.xmask, pack.zmask, pack.coeff, tol)


@dataclass
class CSRRows:
    """Rows `rows` of an operator's CSR (orc_csr_rows): row j of this matrix
    is row rows[j] of the full one; columns are global."""
    n_qubits: int
    rows: np.ndarray     # int64[n]
    rowptr: np.ndarray   # int64[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # complex128[nnz]


def csr_rows(pack, rows, tol: float | None = None) -> CSRRows:
    """Selected rows of the CSR of a Pauli pack (same entries as csr_build)."""
    x = np.ascontiguousarray(pack.xmask, dtype=np.uint64)
    z = np.ascontiguousarray(pack.zmask, dtype=np.uint64)
    c = _c128(pack.coeff)
    if tol is None:
        tol = default_tol(c)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    rowptr = np.zeros(r.size + 1, dtype=np.int64)
    cd = c.view(np.float64)
    nnz = lib().orc_csr_rows(pack.n_qubits, x.size, x, z, cd, tol, r, r.size, rowptr, None, None)
    if nnz < 0:
        raise ValueError("oracle csr_rows: bad arguments")
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    val = np.zeros(max(nnz, 1), dtype=np.complex128)
    lib().orc_csr_rows(pack.n_qubits, x.size, x, z, cd, tol, r, r.size, rowptr,
                       col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p))
    return CSRRows(pack.n_qubits, r, rowptr, col[:nnz], val[:nnz])


def spmv_rows(m: CSRRows, x) -> np.ndarray:
    """(M x)_{rows[j]} for every selected row j (orc_spmv over the row subset)."""
    x = _c128(x)
    y = np.zeros(m.rows.size, dtype=np.complex128)
    col = m.col if m.col.size else np.zeros(1, dtype=np.int32)
    val = np.ascontiguousarray(m.val if m.val.size else np.zeros(1, dtype=np.complex128))
    lib().orc_spmv(m.rows.size, m.rowptr, np.ascontiguousarray(col), val.view(np.float64),
                   x.view(np.float64), y.view(np.float64))
    return y


def _colv(m: CSR):
    col = m.col if m.col.size else np.zeros(1, dtype=np.int32)
    val = m.val if m.val.size else np.zeros(1, dtype=np.complex128)
    return np.ascontiguousarray(col), np.ascontiguousarray(val).view(np.float64)


def spmv(m: CSR, x) -> np.ndarray:
    x = _c128(x)
    y = np.zeros(m.dim, dtype=np.complex128)
    col, val = _colv(m)
    lib().orc_spmv(m.dim, m.rowptr, col, val, x.view(np.float64), y.view(np.float64))
    return y


def taylor5(a: CSR, theta: float, psi) -> np.ndarray:
    """Raw Eq. 8 result (not renormalised)."""
    psi = _c128(psi)
    out = np.zeros_like(psi)
    work = np.zeros(4 * a.dim, dtype=np.float64)
    col, val = _colv(a)
    lib().orc_taylor5(a.dim, a.rowptr, col, val, float(theta), psi.view(np.float64),
                      out.view(np.float64), work)
    return out


def normalize(psi) -> tuple[np.ndarray, float]:
    out = _c128(psi).copy()
    n2 = lib().orc_normalize(out.size, out.view(np.float64))
    return out, float(n2)


def energy(h: CSR, psi):
    """Returns (E, <psi|psi>, Im<psi|H psi>, sigma = H psi)."""
    psi = _c128(psi)
    sigma = np.zeros_like(psi)
    out = np.zeros(3, dtype=np.float64)
    col, val = _colv(h)
    lib().orc_energy(h.dim, h.rowptr, col, val, psi.view(np.float64), sigma.view(np.float64), out)
    return float(out[0]), float(out[1]), float(out[2]), sigma


def gradients(pool: list, psi, sigma) -> np.ndarray:
    """g_j = 2 Re <sigma | A_j psi> for every operator of the pool (CSR list)."""
    psi = _c128(psi)
    sigma = _c128(sigma)
    M = len(pool)
    dim = psi.size
    keep = [_colv(a) for a in pool]
    rp = (C.c_void_p * M)(*[a.rowptr.ctypes.data for a in pool])
    cp = (C.c_void_p * M)(*[k[0].ctypes.data for k in keep])
    vp = (C.c_void_p * M)(*[k[1].ctypes.data for k in keep])
    g = np.zeros(M, dtype=np.float64)
    work = np.zeros(2 * dim, dtype=np.float64)
    lib().orc_gradients(dim, M, rp, cp, vp, psi.view(np.float64), sigma.view(np.float64), g, work)
    return g


def select(g, rel_tie: float = REL_TIE) -> tuple[int, float]:
    g = np.ascontiguousarray(g, dtype=np.float64)
    gm = C.c_double(0.0)
    k = lib().orc_select(g.size, g, rel_tie, C.byref(gm))
    return int(k), float(gm.value)


def step_energy(h: CSR, a: CSR, psi, theta: float) -> float:
    """Energy (Eq. 1) of the state the update of Eq. 6-8 makes from psi with
    generator a and angle theta, after renormalisation."""
    phi, _ = normalize(taylor5(a, float(theta), psi))
    return energy(h, phi)[0]


def minimise_angle(f, theta_max: float, n_grid: int):
    """Minimiser of f over [-theta_max, theta_max]: the best point of a
    uniform grid, refined by a bounded scalar minimisation (Brent's method,
    scipy) on the bracket around it.  Returns (theta, f(theta))."""
    from scipy.optimize import minimize_scalar
    grid = np.linspace(-theta_max, theta_max, n_grid)
    vals = np.array([f(t) for t in grid])
    i = int(np.argmin(vals))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, n_grid - 1)]
    res = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-13})
    if res.fun <= vals[i]:
        return float(res.x), float(res.fun)
    return float(grid[i]), float(vals[i])


def line_search(h: CSR, a: CSR, psi, theta_max: float = 1.0, n_grid: int = 201):
    """The angle in [-theta_max, theta_max] that minimises step_energy (grid,
    then Brent's method on the bracket around the best point).  Returns
    (theta, E)."""
    return minimise_angle(lambda t: step_energy(h, a, psi, t), theta_max, n_grid)


def ansatz_state(pool: list, ref, ks, thetas) -> np.ndarray:
    """The adaptive ansatz: starting from the reference, the update of
    Eq. 6-8 with generator pool[ks[m]] and angle thetas[m] for m = 0, 1, ...
    in order, each followed by renormalisation."""
    psi = _c128(ref).copy()
    for k, t in zip(ks, thetas):
        psi, _ = normalize(taylor5(pool[int(k)], float(t), psi))
    return psi


def ansatz_energy(h: CSR, pool: list, ref, ks, thetas) -> float:
    """Energy (Eq. 1) of the ansatz state."""
    return energy(h, ansatz_state(pool, ref, ks, thetas))[0]


def reoptimize(h: CSR, pool: list, ref, ks, thetas, sweeps: int = 1, theta_max: float = 1.0,
               n_grid: int = 201, trace: list | None = None) -> np.ndarray:
    """Re-optimise every angle of the ansatz by cyclic coordinate descent:
    each sweep visits m = 0, 1, ..., n-1 in order and replaces thetas[m] by
    the minimiser over [-theta_max, theta_max] of ansatz_energy as a function
    of that angle alone, the others held at their current values (the angles
    before m already updated in this sweep).  With ``trace`` each visited
    coordinate appends (m, the angles before the visit, the new angle, its
    energy).  Returns the new angles."""
    th = np.array(thetas, dtype=np.float64).copy()
    for _ in range(sweeps):
        for m in range(len(ks)):
            before = th.copy()

            def f(t, m=m):
                trial = th.copy()
                trial[m] = t
                return ansatz_energy(h, pool, ref, ks, trial)

            t_new, e_new = minimise_angle(f, theta_max, n_grid)
            th[m] = t_new
            if trace is not None:
                trace.append((m, before, t_new, e_new))
    return th


@dataclass
class AdaptTrace:
    energies: list        # energy at psi_t before each update, then the final one
    gradients: list       # g at psi_t
    selected: list        # chosen index k_t
    thetas: list
    psi: np.ndarray       # final state


def adapt_run(h: CSR, pool: list, psi0, thetas, steps: int, renormalize: bool = True,
              forced=None, eps: float = 0.0, line_search_max: float | None = None,
              reopt_sweeps: int = 0) -> AdaptTrace:
    """Adaptive loop (Sec. III-D): screen, select, check convergence, update.

    ``forced`` (optional sequence of indices) replaces the selection, so that
    another implementation can be compared along the same trajectory.  With
    ``line_search_max`` the angle of each update is line_search's minimiser
    over [-line_search_max, line_search_max] instead of thetas[t] (thetas may
    then be None).  With ``reopt_sweeps`` > 0, after each update every angle
    chosen so far is re-optimised (reoptimize, over the same range) and the
    state is rebuilt from psi0; tr.thetas then holds the final angles.
    """
    psi = _c128(psi0).copy()
    tr = AdaptTrace([], [], [], [], psi)
    for t in range(steps):
        e, _, _, sigma = energy(h, psi)
        g = gradients(pool, psi, sigma)
        k, gmax = select(g)
        tr.energies.append(e)
        tr.gradients.append(g)
        if gmax < eps:
            break
        if forced is not None:
            k = int(forced[t])
        tr.selected.append(k)
        if line_search_max is not None:
            theta = line_search(h, pool[k], psi, line_search_max)[0]
        else:
            theta = float(thetas[t])
        tr.thetas.append(theta)
        psi = taylor5(pool[k], theta, psi)
        if renormalize:
            psi, _ = normalize(psi)
        if reopt_sweeps > 0:
            tm = line_search_max if line_search_max is not None else 1.0
            tr.thetas = list(reoptimize(h, pool, psi0, tr.selected, tr.thetas, reopt_sweeps, tm))
            psi = ansatz_state(pool, psi0, tr.selected, tr.thetas)
    tr.energies.append(energy(h, psi)[0])
    tr.psi = psi
    return tr
