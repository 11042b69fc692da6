"""MI355X (gfx950) hot path of the adaptive-VQE simulator.

The compute lives in libadaptvqe.so (HIP, built by ``build.py``); ``binding``
exposes its C ABI (include/adaptvqe.h) with the same names.  ``batch``,
``tune`` and ``serve`` add batched HIP-graph steps, the SpMV schedule
autotuner and the continuous-batching request loop on top.
"""
from .binding import (BatchPlan, Context, DeviceCSR, DevicePool, VqeError, csr_build_from_pauli,
                      csr_from_pack, energy, pool_from_packs, pool_gradients, taylor5_apply,
                      vqe_select)

__all__ = ["BatchPlan", "Context", "DeviceCSR", "DevicePool", "VqeError", "csr_build_from_pauli",
           "csr_from_pack", "energy", "pool_from_packs", "pool_gradients", "taylor5_apply",
           "vqe_select"]
