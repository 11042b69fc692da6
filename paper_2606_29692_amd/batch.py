"""Device-resident systems and batched adaptive steps.

A :class:`DeviceSystem` holds one run on the GPU: its Hamiltonian CSR (FP64,
or FP32 storage with an FP64 diagonal shift), its pool (shared by every run
with the same register size, electron count, mapping and dtype) and its state
vector.  :func:`make_batch` groups systems into one :class:`BatchPlan`, whose
step is a fixed launch sequence that can be replayed as a HIP graph.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import binding as B

_TORCH_DTYPE = {"c128": "complex128", "c64": "complex64"}


def _torch():
    import torch
    return torch


@dataclass
class DeviceSystem:
    key: tuple               # (n_qubits, n_electrons, mapping)
    H: B.DeviceCSR
    pool: B.DevicePool
    psi: object              # torch tensor on the device
    reference_index: int
    dtype: str

    @property
    def n_qubits(self) -> int:
        return self.H.n_qubits

    @property
    def shift(self) -> float:
        return self.H.diag_shift

    def reset(self):
        """Back to the reference determinant."""
        self.psi.zero_()
        self.psi[self.reference_index] = 1.0

    def nbytes(self, include_pool: bool = True) -> int:
        b = self.H.nbytes() + 2 * self.psi.numel() * self.psi.element_size()
        return b + (self.pool.nbytes() if include_pool else 0)


class PoolCache:
    """One device pool per (n_qubits, n_electrons, mapping, dtype).  With
    matrix_free=True the pools are matrix-free (no generator CSR on the
    device; batch plans screen and update from the Pauli-derived records)."""

    def __init__(self, ctx: B.Context, matrix_free: bool = False):
        self.ctx = ctx
        self.matrix_free = matrix_free
        self._pools: dict = {}

    def get(self, key: tuple, packs, dtype: str):
        k = key + (dtype,)
        if k not in self._pools:
            self._pools[k] = (B.MatrixFreePool(packs, dtype) if self.matrix_free
                              else B.pool_from_packs(self.ctx, packs, dtype))
        return self._pools[k]

    def drop(self, key: tuple, dtype: str):
        self._pools.pop(key + (dtype,), None)

    def nbytes(self) -> int:
        return sum(p.nbytes() for p in self._pools.values())


def reference_diagonal(ctx: B.Context, H64: B.DeviceCSR, r: int) -> float:
    """H[r, r] of a device CSR (read back from the device)."""
    torch = _torch()
    lo, hi = (int(v) for v in H64.rowptr[r:r + 2].cpu())
    cols = H64.col[lo:hi].cpu().numpy()
    vals = H64.val[lo:hi].cpu().numpy()
    hit = np.nonzero(cols == r)[0]
    torch.cuda.synchronize()
    return float(vals[hit[0]].real) if hit.size else 0.0


def device_system(ctx: B.Context, system, dtype: str = "c128", pools: PoolCache | None = None
                  ) -> DeviceSystem:
    """Upload a vqe_system.System: CSR build on the device (FP32 storage takes
    the reference determinant's diagonal as its FP64 shift)."""
    torch = _torch()
    spec = system.spec
    key = (spec.n_qubits, spec.n_electrons, spec.mapping)
    H64 = B.csr_from_pack(ctx, system.hamiltonian, "c128")
    if dtype == "c128":
        H = H64
    else:
        shift = reference_diagonal(ctx, H64, system.reference_index)
        H = B.csr_from_pack(ctx, system.hamiltonian, "c64", diag_shift=shift)
        del H64
    pools = pools or PoolCache(ctx)
    pool = pools.get(key, system.pool, dtype)
    psi = torch.zeros(1 << spec.n_qubits, dtype=getattr(torch, _TORCH_DTYPE[dtype]),
                      device=ctx.torch_device)
    psi[system.reference_index] = 1.0
    return DeviceSystem(key, H, pool, psi, system.reference_index, dtype)


def make_batch(ctx: B.Context, systems: list, schedules=None) -> B.BatchPlan:
    return B.BatchPlan(ctx, [(s.H, s.pool, s.psi) for s in systems], schedules=schedules)


def bytes_per_step(systems: list, value_form: str = "complex") -> dict:
    """Algorithmic HBM bytes of one adaptive step (canonical CSR with
    interleaved complex values, each vector once): the H product and the pool
    screen (pool CSR counted once per distinct pool), and the Taylor update of
    a single-excitation generator.  value_form "real" counts the values of an
    operator whose entries are all real at half the complex element (the
    accounting of the real-value specialisation, reported apart from the
    complex contract)."""
    if value_form not in ("complex", "real"):
        raise ValueError(f"value form {value_form!r}")
    out = {"h_spmv": 0, "pool_screen": 0, "taylor": 0}
    seen = set()

    def vsize(op):
        return op.val.element_size() // (2 if value_form == "real" and op.real else 1)

    for s in systems:
        dim = s.H.dim
        sx = s.psi.element_size()
        sv = vsize(s.H)
        out["h_spmv"] += 4 * (dim + 1) + s.H.nnz * (4 + sv) + 2 * dim * sx
        out["pool_screen"] += 2 * dim * sx + 8 * s.pool.M
        if isinstance(s.pool, B.MatrixFreePool):
            # no generator arrays: the update reads and writes the support of
            # a single excitation (2^(N-1) amplitudes)
            out["taylor"] += 2 * (dim // 2) * sx
            continue
        pid = id(s.pool)
        if pid not in seen:
            seen.add(pid)
            out["pool_screen"] += sum(4 * (dim + 1) + o.nnz * (4 + vsize(o)) for o in s.pool.ops)
        single = max(s.pool.ops, key=lambda o: o.nnz)
        out["taylor"] += 4 * (dim + 1) + single.nnz * (4 + vsize(single)) + 2 * dim * sx
    return out


class AnsatzHistory:
    """The generator and angle of every update applied so far to each slot of
    a batch plan (device tensors [B, max_steps]), with each slot's reference
    state, for the re-optimisation of every angle (vqe_batch_reoptimize)."""

    def __init__(self, plan: B.BatchPlan, max_steps: int):
        torch = _torch()
        dev = plan.k.device
        self.plan = plan
        self.ks = torch.full((plan.B, max_steps), -1, dtype=torch.int32, device=dev)
        self.thetas = torch.zeros((plan.B, max_steps), dtype=torch.float64, device=dev)
        self.refs = [psi.clone() for (_, _, psi) in plan.states]
        self.n = 0

    def record(self):
        """Append the plan's last selection and angle (device copies)."""
        if self.n >= self.ks.shape[1]:
            raise ValueError("AnsatzHistory: more updates than max_steps")
        self.ks[:, self.n].copy_(self.plan.k)
        self.thetas[:, self.n].copy_(self.plan.theta)
        self.n += 1

    def reoptimize(self, sweeps: int = 1, theta_max: float = 1.0, energies=None):
        self.plan.reoptimize(self.ks, self.thetas, self.n, self.refs, sweeps, theta_max, energies)
