"""Alg. 1 in the library (host code) against the oracle's greedy colouring:
identical families on random graphs and on the oracle's graphs of whole
pools (JW and BK)."""
import numpy as np
import pytest

import vqe_system as vs
from oracle import partition as P
from paper_2606_29692_amd import binding as B


def test_random_graphs():
    rng = np.random.default_rng(11)
    for _ in range(40):
        M = int(rng.integers(1, 60))
        a = rng.random((M, M)) < rng.uniform(0.0, 0.7)
        adj = np.triu(a, 1)
        adj = adj | adj.T
        np.testing.assert_array_equal(B.partition_greedy(adj), P.greedy_partition(adj))


@pytest.mark.parametrize("n,ne,mapping", [(8, 4, "jw"), (8, 4, "bk"), (12, 8, "jw")])
def test_pool_graphs(n, ne, mapping):
    s = vs.make_system(vs.SystemSpec(n, ne, mapping, False, 12))
    adj = P.noncommutation_graph(s.pool)
    fam = B.partition_greedy(adj)
    np.testing.assert_array_equal(fam, P.greedy_partition(adj))
