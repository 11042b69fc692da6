"""Thin ctypes binding of libadaptvqe (include/adaptvqe.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch
provides device memory (tensors) and streams.  The functions keep the C names:
``csr_build_from_pauli``, ``taylor5_apply``, ``energy``, ``pool_gradients``,
``vqe_select`` and the batch plan.  If the library is missing or no GPU is
visible, the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libadaptvqe.so")

VQE_OK, VQE_EINVAL, VQE_ESIZE, VQE_ENOMEM, VQE_EHIP, VQE_ENOTSUP = 0, -1, -2, -3, -4, -5
VQE_C128, VQE_C64 = 0, 1
VQE_PAIRING = 1
VQE_REAL = 2
VQE_STEP_RENORM, VQE_STEP_FORCED, VQE_STEP_NO_UPDATE, VQE_STEP_GRAPH = 1, 2, 4, 8
VQE_STEP_LINESEARCH = 16
VQE_STEP_TILED_SCREEN = 32
VQE_SPMV_VEC4 = 0x100
VQE_SPMV_LDS = 0x200
VQE_SPMV_DEEP = 0x400
VQE_SPMV_PREFETCH = 0x800
VQE_SPMV_X16 = 0x4000
VQE_SPMV_REAL = 0x8000
VQE_SPMV_PAD = 0x10000
VQE_SPMV_SLICED = 0x40000
VQE_SPMV_XIDX = 0x80000
REL_TIE = 1e-6

DTYPES = {"c128": VQE_C128, "c64": VQE_C64}


class VqeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


# Injected failures, for tests of failure handling: kind -> failures left.
# "alloc": the binding's next device allocations raise VqeError(VQE_ENOMEM)
# before touching the device, as the library reports a failed allocation.
# The environment variable ADAPTVQE_FAULT=alloc:N arms N of them at import.
_FAULTS: dict = {}
_FAULT_STATUS = {"alloc": VQE_ENOMEM}


def inject_fault(kind: str, count: int = 1):
    if kind not in _FAULT_STATUS:
        raise ValueError(f"unknown fault kind {kind!r}")
    _FAULTS[kind] = int(count)


def check_fault(kind: str):
    """Raise the injected failure of this kind if one is armed."""
    n = _FAULTS.get(kind, 0)
    if n > 0:
        _FAULTS[kind] = n - 1
        raise VqeError(_FAULT_STATUS[kind], f"injected {kind} failure")


def _arm_from_env():
    spec = os.environ.get("ADAPTVQE_FAULT", "")
    if spec:
        kind, _, n = spec.partition(":")
        inject_fault(kind, int(n or 1))


_arm_from_env()


class vqe_csr(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("dtype", C.c_int32), ("dim", C.c_int64),
                ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("diag_shift", C.c_double), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]


VQE_MF_MAX_CON = 8


class vqe_mf_desc(C.Structure):
    _fields_ = [("x", C.c_uint64), ("zsign", C.c_uint64), ("v_re", C.c_double),
                ("v_im", C.c_double), ("n_qubits", C.c_int32), ("n_con", C.c_int32),
                ("beta", C.c_uint64 * VQE_MF_MAX_CON), ("kbits", C.c_uint32),
                ("reserved", C.c_uint32)]


class vqe_pool(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_qubits", C.c_int32), ("dtype", C.c_int32),
                ("all_pairing", C.c_int32), ("ops", C.c_void_p), ("ops_host", C.c_void_p),
                ("mf", C.c_void_p)]


class vqe_batch_item(C.Structure):
    _fields_ = [("H", C.c_void_p), ("pool", C.c_void_p), ("psi", C.c_void_p),
                ("sigma", C.c_void_p), ("spmv_schedule", C.c_int32), ("reserved", C.c_int32)]


class vqe_batch_io(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("energy_out", C.c_void_p), ("g_out", C.c_void_p),
                ("g_offset_host", C.c_void_p), ("k_io", C.c_void_p), ("gmax_out", C.c_void_p),
                ("active", C.c_void_p)]


# name -> (restype, argtypes); the full exported surface of adaptvqe.h
SIGNATURES = {
    "vqe_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "vqe_destroy": (C.c_int, [C.c_void_p]),
    "vqe_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vqe_strerror": (C.c_char_p, [C.c_int]),
    "vqe_last_error": (C.c_char_p, [C.c_void_p]),
    "vqe_device_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_char_p, C.c_int32]),
    "csr_build_from_pauli": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_double, C.c_int32, C.c_double,
                                       C.POINTER(vqe_csr), C.POINTER(C.c_int64)]),
    "taylor5_apply": (C.c_int, [C.c_void_p, C.POINTER(vqe_csr), C.c_double, C.c_void_p,
                                C.c_int32, C.c_void_p]),
    "energy": (C.c_int, [C.c_void_p, C.POINTER(vqe_csr), C.c_void_p, C.c_void_p, C.c_void_p]),
    "energy_noalloc": (C.c_int, [C.c_void_p, C.POINTER(vqe_csr), C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "pool_gradients": (C.c_int, [C.c_void_p, C.POINTER(vqe_csr), C.POINTER(vqe_pool),
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "vqe_select": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_void_p,
                             C.c_void_p]),
    "vqe_batch_create": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(vqe_batch_item),
                                   C.POINTER(vqe_batch_io), C.c_double, C.POINTER(C.c_void_p)]),
    "vqe_batch_step": (C.c_int, [C.c_void_p, C.c_uint32]),
    "vqe_batch_rebind": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(vqe_batch_item)]),
    "vqe_batch_step_timed": (C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p), C.c_int32]),
    "vqe_batch_run": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_int32]),
    "vqe_batch_destroy": (C.c_int, [C.c_void_p]),
    "vqe_batch_set_line_search": (C.c_int, [C.c_void_p, C.c_double]),
    "vqe_batch_reoptimize": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                       C.c_void_p, C.c_int32, C.c_double, C.c_void_p]),
    "vqe_batch_workspace_bytes": (C.c_int64, [C.c_void_p]),
    "vqe_batch_time_products": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_float)]),
    "vqe_batch_layout_entries": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    "vqe_layout_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "vqe_layout_destroy": (C.c_int, [C.c_void_p]),
    "vqe_layout_bytes": (C.c_int64, [C.c_void_p]),
    "vqe_batch_rebind_layout": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "vqe_time_spmv": (C.c_int, [C.c_void_p, C.POINTER(vqe_csr), C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_int32, C.POINTER(C.c_float)]),
    "vqe_default_schedule": (C.c_int32, [C.POINTER(vqe_csr)]),
    "vqe_mf_describe": (C.c_int, [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_double, C.POINTER(vqe_mf_desc)]),
    "vqe_mf_pool_create": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "vqe_mf_pool_destroy": (C.c_int, [C.c_void_p]),
    "vqe_mf_pool_get": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(vqe_mf_desc)]),
    "vqe_mf_owner_rows": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                    C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "vqe_mf_noncommutation": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "vqe_partition_greedy": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
}

_lib = None


def lib():
    """Load libadaptvqe.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2606_29692_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the adaptvqe HIP path needs an MI355X")
    return torch


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


class Context:
    """A vqe_ctx bound to one device and one stream (torch's current stream
    unless given)."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        st = lib().vqe_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != VQE_OK:
            raise VqeError(st, f"vqe_create: {lib().vqe_strerror(st).decode()}")
        self.handle = h
        # batch plans and sliced layouts made on this context: destroyed
        # before the context, since they use its stream until destroyed
        self._plans = weakref.WeakSet()

    def check(self, status: int, what: str):
        if status != VQE_OK:
            msg = lib().vqe_last_error(self.handle).decode()
            raise VqeError(status, f"{what}: {lib().vqe_strerror(status).decode()}: {msg}")

    def set_stream(self, stream):
        self.stream = stream
        self.check(lib().vqe_set_stream(self.handle, C.c_void_p(stream.cuda_stream)), "vqe_set_stream")

    def info(self):
        n = C.c_int32()
        buf = C.create_string_buffer(256)
        self.check(lib().vqe_device_info(self.handle, C.byref(n), buf, 256), "vqe_device_info")
        return int(n.value), buf.value.decode()

    def close(self):
        if getattr(self, "handle", None):
            for plan in list(getattr(self, "_plans", ())):
                plan.close()
            lib().vqe_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceCSR:
    """A CSR operator in device memory (torch tensors) and its vqe_csr descriptor."""

    def __init__(self, desc: vqe_csr, rowptr, col, val):
        self.desc = desc
        self.rowptr, self.col, self.val = rowptr, col, val

    @property
    def nnz(self) -> int:
        return int(self.desc.nnz)

    @property
    def dim(self) -> int:
        return int(self.desc.dim)

    @property
    def n_qubits(self) -> int:
        return int(self.desc.n_qubits)

    @property
    def pairing(self) -> bool:
        return bool(self.desc.flags & VQE_PAIRING)

    @property
    def real(self) -> bool:
        """Every entry is real (set by the builder from the terms)."""
        return bool(self.desc.flags & VQE_REAL)

    @property
    def diag_shift(self) -> float:
        return float(self.desc.diag_shift)

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.rowptr, self.col, self.val))


def default_tol(coeff) -> float:
    coeff = np.asarray(coeff)
    return 1e-12 * float(np.abs(coeff).max()) if coeff.size else 0.0


def csr_build_from_pauli(ctx: Context, n_qubits: int, xmask, zmask, coeff,
                         drop_tol: float | None = None, dtype: str = "c128",
                         diag_shift: float = 0.0) -> DeviceCSR:
    """Compile sum_t coeff[t] P(xmask[t], zmask[t]) to a device CSR (two phases)."""
    torch = _torch()
    x = np.ascontiguousarray(xmask, dtype=np.uint64)
    z = np.ascontiguousarray(zmask, dtype=np.uint64)
    c = np.ascontiguousarray(np.asarray(coeff, dtype=np.complex128))
    if drop_tol is None:
        drop_tol = default_tol(c)
    dt = DTYPES[dtype]
    dim = 1 << n_qubits
    check_fault("alloc")
    rowptr = torch.empty(dim + 1, dtype=torch.int32, device=ctx.torch_device)
    desc = vqe_csr()
    desc.rowptr = rowptr.data_ptr()
    nnz = C.c_int64()
    args = (ctx.handle, n_qubits, x.size, x.ctypes.data, z.ctypes.data, c.ctypes.data,
            float(drop_tol), dt, float(diag_shift))
    ctx.check(lib().csr_build_from_pauli(*args, C.byref(desc), C.byref(nnz)),
              "csr_build_from_pauli (sizing)")
    n = max(int(nnz.value), 1)
    check_fault("alloc")
    col = torch.empty(n, dtype=torch.int32, device=ctx.torch_device)
    val = torch.empty(n, dtype=torch.complex128 if dt == VQE_C128 else torch.complex64,
                      device=ctx.torch_device)
    desc.col = col.data_ptr()
    desc.val = val.data_ptr()
    ctx.check(lib().csr_build_from_pauli(*args, C.byref(desc), C.byref(nnz)),
              "csr_build_from_pauli (fill)")
    return DeviceCSR(desc, rowptr, col, val)


def csr_from_pack(ctx: Context, pack, dtype: str = "c128", diag_shift: float = 0.0,
                  drop_tol: float | None = None) -> DeviceCSR:
    return csr_build_from_pauli(ctx, pack.n_qubits, pack.xmask, pack.zmask, pack.coeff,
                                drop_tol, dtype, diag_shift)


def taylor5_apply(ctx: Context, A: DeviceCSR, theta: float, psi, renormalize: bool = True,
                  norm2_out=None):
    """In-place fifth-order Taylor update of psi (Eq. 6-8)."""
    ctx.check(lib().taylor5_apply(ctx.handle, C.byref(A.desc), float(theta), _ptr(psi),
                                  1 if renormalize else 0, _ptr(norm2_out)), "taylor5_apply")
    return psi


def energy(ctx: Context, H: DeviceCSR, psi, sigma_out=None, out=None):
    """out (device double[3]) = (E, <psi|psi>, Im<psi|S psi>); sigma_out = S psi."""
    torch = _torch()
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().energy(ctx.handle, C.byref(H.desc), _ptr(psi), _ptr(sigma_out), _ptr(out)),
              "energy")
    return out


VQE_NOALLOC_SCRATCH_BYTES = 4 << 20


def energy_noalloc(ctx: Context, H: DeviceCSR, psi, sigma_out, out):
    """energy() without any device allocation: sigma_out and out (device
    double[3]) are the caller's; the reduction's partial sums use the
    library's static per-GPU scratch array (see the header)."""
    ctx.check(lib().energy_noalloc(ctx.handle, C.byref(H.desc), _ptr(psi), _ptr(sigma_out),
                                   _ptr(out)), "energy_noalloc")
    return out


class DevicePool:
    """M generators (DeviceCSR) and their device descriptor table."""

    def __init__(self, ctx: Context, ops: list):
        torch = _torch()
        if not ops:
            raise ValueError("empty pool")
        self.ops = ops
        M = len(ops)
        self._host = (vqe_csr * M)(*[o.desc for o in ops])
        raw = np.frombuffer(C.string_at(C.addressof(self._host), C.sizeof(self._host)), dtype=np.uint8)
        self._dev = torch.from_numpy(raw.copy()).to(ctx.torch_device)
        d0 = ops[0].desc
        self.desc = vqe_pool()
        self.desc.M = M
        self.desc.n_qubits = d0.n_qubits
        self.desc.dtype = d0.dtype
        self.desc.all_pairing = int(all(o.pairing for o in ops))
        self.desc.ops = self._dev.data_ptr()
        self.desc.ops_host = C.addressof(self._host)

    @property
    def M(self) -> int:
        return len(self.ops)

    def nbytes(self) -> int:
        return sum(o.nbytes() for o in self.ops) + self._dev.numel()


def pool_from_packs(ctx: Context, packs, dtype: str = "c128") -> DevicePool:
    return DevicePool(ctx, [csr_from_pack(ctx, p, dtype) for p in packs])


# ---------------------------------------------------------------- matrix-free generators
def _desc_dict(d: vqe_mf_desc) -> dict:
    return {"x": int(d.x), "zsign": int(d.zsign), "v": complex(d.v_re, d.v_im),
            "n_qubits": int(d.n_qubits), "beta": [int(d.beta[i]) for i in range(d.n_con)],
            "kbits": int(d.kbits)}


def _pack_arrays(packs):
    xs, zs, cs, off = [], [], [], [0]
    for p in packs:
        xs.append(np.asarray(p.xmask, dtype=np.uint64))
        zs.append(np.asarray(p.zmask, dtype=np.uint64))
        c = np.asarray(p.coeff, dtype=np.complex128)
        cs.append(np.ascontiguousarray(np.stack([c.real, c.imag], axis=1)).reshape(-1))
        off.append(off[-1] + len(c))
    return (np.ascontiguousarray(np.concatenate(xs)), np.ascontiguousarray(np.concatenate(zs)),
            np.ascontiguousarray(np.concatenate(cs)), np.asarray(off, dtype=np.int64))


def mf_describe(pack, drop_tol: float | None = None) -> dict:
    """Matrix-free form of one generator (host computation, no GPU): the
    flip mask x, sign mask zsign, value v and support constraints
    (|beta_i & c| mod 2 = bit i of kbits).  Raises VqeError when the
    generator has no such form."""
    x, z, c, _ = _pack_arrays([pack])
    if drop_tol is None:
        drop_tol = default_tol(pack.coeff)
    d = vqe_mf_desc()
    rc = lib().vqe_mf_describe(int(pack.n_qubits), len(x), x.ctypes.data, z.ctypes.data,
                               c.ctypes.data, float(drop_tol), C.byref(d))
    if rc != 0:
        raise VqeError(rc, f"vqe_mf_describe: {lib().vqe_strerror(rc).decode()}")
    return _desc_dict(d)


class MfPool:
    """A pool in matrix-free form (host descriptors; no GPU needed to build)."""

    def __init__(self, packs, drop_tol=None):
        packs = list(packs)
        if not packs:
            raise ValueError("empty pool")
        x, z, c, off = _pack_arrays(packs)
        tol = None
        if drop_tol is not None:
            tol = np.ascontiguousarray(np.broadcast_to(np.asarray(drop_tol, dtype=np.float64),
                                                       (len(packs),)))
        h = C.c_void_p()
        rc = lib().vqe_mf_pool_create(int(packs[0].n_qubits), len(packs), off.ctypes.data,
                                      x.ctypes.data, z.ctypes.data, c.ctypes.data,
                                      tol.ctypes.data if tol is not None else None, C.byref(h))
        if rc != 0:
            raise VqeError(rc, f"vqe_mf_pool_create: {lib().vqe_strerror(rc).decode()}")
        self.handle = h.value
        self.M = len(packs)
        self.n_qubits = int(packs[0].n_qubits)

    def get(self, j: int) -> dict:
        d = vqe_mf_desc()
        rc = lib().vqe_mf_pool_get(self.handle, int(j), C.byref(d))
        if rc != 0:
            raise VqeError(rc, "vqe_mf_pool_get")
        return _desc_dict(d)

    def owner_rows(self, j: int, tile_rows: int, tile: int = -1):
        """(rows, tile indices) of generator j on one screen tile (tile = -1:
        the whole state), in the device's enumeration order."""
        n = C.c_int64()
        rc = lib().vqe_mf_owner_rows(self.handle, int(j), int(tile_rows), int(tile), C.byref(n),
                                     None, None)
        if rc != 0:
            raise VqeError(rc, "vqe_mf_owner_rows")
        rows = np.zeros(n.value, dtype=np.uint32)
        idx = np.zeros(n.value, dtype=np.uint32)
        rc = lib().vqe_mf_owner_rows(self.handle, int(j), int(tile_rows), int(tile), C.byref(n),
                                     rows.ctypes.data, idx.ctypes.data)
        if rc != 0:
            raise VqeError(rc, "vqe_mf_owner_rows")
        return rows, idx

    def close(self):
        if getattr(self, "handle", None):
            lib().vqe_mf_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def noncommutation_graph(ctx: "Context", pool: "MfPool"):
    """Alg. 1's complementary graph on the device: bool M x M (host copy)."""
    torch = _torch()
    adj = torch.empty(pool.M * pool.M, dtype=torch.uint8, device=ctx.torch_device)
    ctx.check(lib().vqe_mf_noncommutation(ctx.handle, pool.handle, adj.data_ptr()),
              "vqe_mf_noncommutation")
    return adj.cpu().numpy().reshape(pool.M, pool.M).astype(bool)


def partition_greedy(adj) -> np.ndarray:
    """Alg. 1 (host): family index of every vertex of a boolean adjacency matrix."""
    a = np.ascontiguousarray(np.asarray(adj, dtype=np.uint8))
    M = a.shape[0]
    fam = np.zeros(M, dtype=np.int32)
    nf = C.c_int32()
    rc = lib().vqe_partition_greedy(M, a.ctypes.data, fam.ctypes.data, C.byref(nf))
    if rc != 0:
        raise VqeError(rc, "vqe_partition_greedy")
    return fam


class MatrixFreePool:
    """A pool for batch plans that is applied from its matrix-free form only:
    no generator CSR exists on the device."""

    def __init__(self, packs, dtype: str = "c128", drop_tol=None):
        self.mf = MfPool(packs, drop_tol)
        self.desc = vqe_pool()
        self.desc.M = self.mf.M
        self.desc.n_qubits = self.mf.n_qubits
        self.desc.dtype = DTYPES[dtype]
        self.desc.all_pairing = 1
        self.desc.ops = None
        self.desc.ops_host = None
        self.desc.mf = self.mf.handle

    @property
    def M(self) -> int:
        return self.mf.M

    @property
    def ops(self) -> list:
        return []

    def nbytes(self) -> int:
        return 0


def pool_gradients(ctx: Context, H: DeviceCSR, pool: DevicePool, psi, sigma=None, g_out=None):
    """g_j = 2 Re <H psi | A_j psi> for every generator (Eq. 5); device double[M]."""
    torch = _torch()
    if g_out is None:
        g_out = torch.empty(pool.M, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().pool_gradients(ctx.handle, C.byref(H.desc), C.byref(pool.desc), _ptr(psi),
                                   _ptr(sigma), _ptr(g_out)), "pool_gradients")
    return g_out


def vqe_select(ctx: Context, g, rel_tie: float = REL_TIE, k_out=None, gmax_out=None):
    """Index of the largest |g_j| (lowest index within rel_tie); device tensors."""
    torch = _torch()
    if k_out is None:
        k_out = torch.empty(1, dtype=torch.int32, device=ctx.torch_device)
    if gmax_out is None:
        gmax_out = torch.empty(1, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().vqe_select(ctx.handle, int(g.numel()), _ptr(g), float(rel_tie), _ptr(k_out),
                               _ptr(gmax_out)), "vqe_select")
    return k_out, gmax_out


def time_spmv(ctx: Context, H: DeviceCSR, psi, sigma, schedule: int, reps: int = 20) -> float:
    ms = C.c_float()
    ctx.check(lib().vqe_time_spmv(ctx.handle, C.byref(H.desc), _ptr(psi), _ptr(sigma), int(schedule),
                                  int(reps), C.byref(ms)), "vqe_time_spmv")
    return float(ms.value)


def default_schedule(H: DeviceCSR) -> int:
    return int(lib().vqe_default_schedule(C.byref(H.desc)))


class Layout:
    """A sliced layout of one operator for a batch schedule (vqe_layout_create),
    to be bound to plan slots with BatchPlan.rebind(..., layout=...)."""

    def __init__(self, ctx: Context, H: DeviceCSR, schedule: int):
        h = C.c_void_p()
        ctx.check(lib().vqe_layout_create(ctx.handle, C.addressof(H.desc), int(schedule), C.byref(h)),
                  "vqe_layout_create")
        self.ctx, self.H, self.handle = ctx, H, h
        ctx._plans.add(self)

    def nbytes(self) -> int:
        return int(lib().vqe_layout_bytes(self.handle)) if self.handle else 0

    def close(self):
        if self.handle:
            if getattr(self.ctx, "handle", None):     # as BatchPlan.close
                lib().vqe_layout_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """One adaptive step for B states per launch sequence (optionally a HIP graph).

    ``states`` is a list of (H: DeviceCSR, pool: DevicePool, psi tensor) and the
    plan allocates sigma, theta, energies, gradients, indices and gmax as torch
    tensors that stay alive with it."""

    def __init__(self, ctx: Context, states: list, schedules=None, rel_tie: float = REL_TIE,
                 with_active: bool = False):
        torch = _torch()
        self.ctx = ctx
        ctx._plans.add(self)
        B = len(states)
        self.B = B
        self.states = states
        dev = ctx.torch_device
        self.sigma = [torch.empty_like(psi) for (_, _, psi) in states]
        self.g_offset = np.zeros(B, dtype=np.int64)
        off = 0
        for s, (_, pool, _) in enumerate(states):
            self.g_offset[s] = off
            off += pool.M
        self.theta = torch.zeros(B, dtype=torch.float64, device=dev)
        self.energies = torch.zeros(3 * B, dtype=torch.float64, device=dev)
        self.g = torch.zeros(max(off, 1), dtype=torch.float64, device=dev)
        self.k = torch.zeros(B, dtype=torch.int32, device=dev)
        self.gmax = torch.zeros(B, dtype=torch.float64, device=dev)
        # per-slot activity flags (continuous batching); all on by default
        self.active = torch.ones(B, dtype=torch.int32, device=dev) if with_active else None
        self.schedules = schedules
        items = (vqe_batch_item * B)()
        for s, (H, pool, psi) in enumerate(states):
            items[s].H = C.addressof(H.desc)
            items[s].pool = C.addressof(pool.desc)
            items[s].psi = psi.data_ptr()
            items[s].sigma = self.sigma[s].data_ptr()
            items[s].spmv_schedule = int(schedules[s]) if schedules is not None else 0
        self._items = items
        io = vqe_batch_io()
        io.theta = self.theta.data_ptr()
        io.energy_out = self.energies.data_ptr()
        io.g_out = self.g.data_ptr()
        io.g_offset_host = self.g_offset.ctypes.data
        io.k_io = self.k.data_ptr()
        io.gmax_out = self.gmax.data_ptr()
        io.active = self.active.data_ptr() if self.active is not None else None
        self._io = io
        h = C.c_void_p()
        ctx.check(lib().vqe_batch_create(ctx.handle, B, items, C.byref(io), float(rel_tie),
                                         C.byref(h)), "vqe_batch_create")
        self.handle = h

    @staticmethod
    def _flags(renorm, forced, update, graph, line_search, tiled_screen=False):
        return ((VQE_STEP_RENORM if renorm else 0) | (VQE_STEP_FORCED if forced else 0)
                | (0 if update else VQE_STEP_NO_UPDATE) | (VQE_STEP_GRAPH if graph else 0)
                | (VQE_STEP_LINESEARCH if line_search else 0)
                | (VQE_STEP_TILED_SCREEN if tiled_screen else 0))

    def set_line_search(self, theta_max: float):
        """Enable (theta_max > 0) or disable steps whose angle is chosen by line
        search (see vqe_batch_set_line_search); the chosen angles land in theta."""
        self.ctx.check(lib().vqe_batch_set_line_search(self.handle, float(theta_max)),
                       "vqe_batch_set_line_search")

    def reoptimize(self, ks, thetas, n: int, refs: list, sweeps: int = 1,
                   theta_max: float = 1.0, energies=None):
        """Re-optimise every angle of each slot's ansatz (vqe_batch_reoptimize).
        ks: device int32 [B, ld] generator indices; thetas: device float64
        [B, ld] angles, updated in place; n: updates per slot; refs: B device
        tensors (reference states); energies: optional device float64 [B]."""
        torch = _torch()
        if ks.dtype != torch.int32 or thetas.dtype != torch.float64 or ks.dim() != 2 or \
                thetas.shape != ks.shape or ks.shape[0] != self.B or not ks.is_contiguous() or \
                not thetas.is_contiguous() or len(refs) != self.B or not 0 <= n <= ks.shape[1]:
            raise ValueError("reoptimize: ks and thetas must be contiguous [B, ld] int32 / "
                             "float64 device tensors with n <= ld, and refs one per slot")
        if energies is not None and (energies.dtype != torch.float64 or energies.numel() < self.B):
            raise ValueError("reoptimize: energies must be a float64 device tensor of B entries")
        for r, (_, _, psi) in zip(refs, self.states):
            if r.dtype != psi.dtype or r.numel() != psi.numel() or not r.is_contiguous():
                raise ValueError("reoptimize: each reference must match its slot's state")
        ptrs = (C.c_void_p * self.B)(*[r.data_ptr() for r in refs])
        self.ctx.check(lib().vqe_batch_reoptimize(
            self.handle, ks.data_ptr(), thetas.data_ptr(), int(ks.shape[1]), int(n), ptrs,
            int(sweeps), float(theta_max), energies.data_ptr() if energies is not None else None),
            "vqe_batch_reoptimize")

    def step(self, renorm: bool = True, forced: bool = False, update: bool = True,
             graph: bool = False, line_search: bool = False, tiled_screen: bool = False):
        flags = self._flags(renorm, forced, update, graph, line_search, tiled_screen)
        self.ctx.check(lib().vqe_batch_step(self.handle, flags), "vqe_batch_step")

    def run(self, theta_rows=None, renorm: bool = True, forced: bool = False, graph: bool = True,
            tiled_screen: bool = False, line_search_steps: int = 0):
        """Several adaptive steps in one call (vqe_batch_run): theta_rows.shape[0]
        steps, step i taking its angles from row i of theta_rows (a contiguous
        float64 [n_steps, B] tensor on the plan's device), or, with theta_rows
        None, line_search_steps steps that choose their angles by line search;
        with graph the steps are one graph launch."""
        torch = _torch()
        if theta_rows is None:
            if line_search_steps < 0:
                raise ValueError("run: line_search_steps must be >= 0")
            flags = self._flags(renorm, forced, True, graph, True, tiled_screen)
            self.ctx.check(lib().vqe_batch_run(self.handle, flags, None, int(line_search_steps)),
                           "vqe_batch_run")
            return
        if line_search_steps or theta_rows.dtype != torch.float64 or theta_rows.dim() != 2 or \
                theta_rows.shape[1] != self.B or not theta_rows.is_contiguous() or \
                theta_rows.device != self.theta.device:
            raise ValueError("run: theta_rows must be a contiguous float64 [n_steps, B] tensor "
                             "on the plan's device (and no line search with given angles)")
        flags = self._flags(renorm, forced, True, graph, False, tiled_screen)
        self.ctx.check(lib().vqe_batch_run(self.handle, flags, theta_rows.data_ptr(),
                                           int(theta_rows.shape[0])), "vqe_batch_run")

    def step_timed(self, events, renorm: bool = True, forced: bool = False, update: bool = True,
                   graph: bool = False, line_search: bool = False, tiled_screen: bool = False):
        """Step recording 3 or 7 torch.cuda.Event objects on the context stream
        (see vqe_batch_step_timed)."""
        flags = self._flags(renorm, forced, update, graph, line_search, tiled_screen)
        for e in events:
            if not e.cuda_event:          # torch creates the HIP event on first record
                e.record(self.ctx.stream)
        n = len(events)
        arr = (C.c_void_p * n)(*[C.c_void_p(e.cuda_event) for e in events])
        self.ctx.check(lib().vqe_batch_step_timed(self.handle, flags, arr, n), "vqe_batch_step_timed")

    def time_products(self, reps: int = 20) -> float:
        """Average milliseconds of the H products alone over `reps`
        back-to-back launches (see vqe_batch_time_products)."""
        ms = C.c_float()
        self.ctx.check(lib().vqe_batch_time_products(self.handle, int(reps), C.byref(ms)),
                       "vqe_batch_time_products")
        return float(ms.value)

    def layout_entries(self, slot: int) -> int:
        """Entries (pads included) of the slot's sliced layout, else 0."""
        n = C.c_int64()
        self.ctx.check(lib().vqe_batch_layout_entries(self.handle, int(slot), C.byref(n)),
                       "vqe_batch_layout_entries")
        return int(n.value)

    def rebind(self, slot: int, H: DeviceCSR, pool: DevicePool, psi, layout: "Layout | None" = None):
        """Bind another state (same size, dtype, pool) to a slot; the slot keeps
        its sigma buffer.  With `layout` (built for H and this slot's schedule)
        the slot points to it instead of rebuilding its own layout of H."""
        it = vqe_batch_item()
        it.H = C.addressof(H.desc)
        it.pool = C.addressof(pool.desc)
        it.psi = psi.data_ptr()
        it.sigma = self.sigma[slot].data_ptr()
        it.spmv_schedule = int(self.schedules[slot]) if self.schedules is not None else 0
        if layout is None:
            self.ctx.check(lib().vqe_batch_rebind(self.handle, int(slot), C.byref(it)),
                           "vqe_batch_rebind")
        else:
            self.ctx.check(lib().vqe_batch_rebind_layout(self.handle, int(slot), C.byref(it),
                                                         layout.handle), "vqe_batch_rebind_layout")
        # keep the bound objects alive while the slot refers to them
        self._bound = getattr(self, "_bound", {})
        self._bound[slot] = (H, pool, psi, layout)

    def gradients(self, s: int):
        M = self.states[s][1].M
        o = int(self.g_offset[s])
        return self.g[o:o + M]

    def workspace_bytes(self) -> int:
        return int(lib().vqe_batch_workspace_bytes(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            # a context closed first (finalisers of a garbage cycle run in any
            # order, after its weak references are cleared) has taken its
            # stream: the plan is then left to the process's end
            if getattr(self.ctx, "handle", None):
                lib().vqe_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
