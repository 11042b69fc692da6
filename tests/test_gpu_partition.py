"""The device non-commutation graph of matrix-free pools equals the oracle's
(Pauli algebra) bit for bit, and so do the families of Alg. 1."""
import time

import numpy as np
import pytest

import vqe_system as vs
from oracle import partition as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2606_29692_amd import binding as B  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,ne,mapping,stretched", [(8, 4, "jw", False), (8, 4, "bk", False),
                                                    (12, 8, "jw", True), (12, 8, "bk", False),
                                                    (14, 6, "jw", False)])
def test_graph_and_families_match_oracle(ctx, n, ne, mapping, stretched):
    s = vs.make_system(vs.SystemSpec(n, ne, mapping, stretched, 51))
    pool = B.MfPool(s.pool)
    t0 = time.perf_counter()
    adj = B.noncommutation_graph(ctx, pool)
    dt = time.perf_counter() - t0
    ref = P.noncommutation_graph(s.pool)
    print(f"N={n} {mapping}: M={pool.M}, {int(adj.sum()) // 2} non-commuting pairs, "
          f"device graph {dt * 1e3:.1f} ms")
    np.testing.assert_array_equal(adj, ref)
    np.testing.assert_array_equal(B.partition_greedy(adj), P.greedy_partition(ref))
    pool.close()
