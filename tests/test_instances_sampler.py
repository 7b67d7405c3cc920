"""The App. A random binary-TT graph sampler (instances.binary_tt_adjacency), CPU.

Checks, for several (d, r): the TT cores contract (oracle's dense TT matrix) to
the adjacency built independently by following the path states; the graph is
simple (0/1, symmetric, zero diagonal) with at least one edge; its TT rank is
exactly r (App. A, the set S_r with the rejection step); sampling is
reproducible for a seed and a positive bias gives denser graphs on average."""
import numpy as np
import pytest

import instances as I
from oracle import tt


@pytest.mark.parametrize("d,r", [(2, 1), (3, 2), (5, 1), (5, 3), (6, 4), (7, 5)])
def test_sampler_graph_properties(d, r):
    g = I.binary_tt_adjacency(d, r, seed=100 + 7 * d + r)
    A = g.dense
    assert np.array_equal(tt.full_mat(g.cores).round(12), A)
    assert set(np.unique(A)) <= {0.0, 1.0}
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 0) and A.sum() > 0
    assert max(I.tt_matrix_ranks(g.cores)) == r


def test_sampler_reproducible_and_bias():
    a = I.binary_tt_adjacency(6, 3, seed=5)
    b = I.binary_tt_adjacency(6, 3, seed=5)
    assert np.array_equal(a.dense, b.dense)
    dens = lambda bias: np.mean([I.binary_tt_adjacency(6, 3, seed=s, bias=bias).dense.mean() for s in range(12)])
    assert dens(1.0) > dens(0.0)
