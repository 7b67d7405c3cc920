"""Pins of the instance generators and the TT encodings of Sec. 4 (CPU)."""
import numpy as np
import pytest

import instances as I
from oracle import problems as P, tt


def _vectt_dense(A, d):
    n = 2 ** d
    idx = np.zeros((n, n), dtype=np.int64)
    for r in range(n):
        for c in range(n):
            v = 0
            for k in range(d):
                v = v * 4 + 2 * ((r >> (d - 1 - k)) & 1) + ((c >> (d - 1 - k)) & 1)
            idx[r, c] = v
    out = np.zeros(n * n)
    out[idx.reshape(-1)] = A.reshape(-1)
    return out, idx


GRAPHS = [I.grid_4x8(), I.kron_sum_products(6, 4, 2), I.hypercube(5), I.signed_kron(5, 6, 4),
          I.kron_sum_noise(6, 5), I.complete(4), I.odd_cycle_plus_isolated(3), I.odd_cycle_plus_isolated(5),
          I.c5_plus_3k1()]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_generator_tt_equals_independent_dense(g):
    D = tt.full_mat(g.cores)
    assert np.allclose(D, g.dense, atol=1e-12 * max(1.0, np.abs(g.dense).max()))
    assert np.allclose(D, D.T, atol=1e-12 * max(1.0, np.abs(D).max()))


def test_grid_vertex_order_and_edges():
    g = I.grid_4x8()
    A = g.dense
    assert A.sum() == 2 * 52
    assert A[8 * 1 + 2, 8 * 1 + 3] == 1 and A[8 * 1 + 2, 8 * 2 + 2] == 1 and A[7, 8] == 0


def test_config_sizes():
    assert I.config("maxcut_grid_d5")["graph"].d == 5
    assert I.config("maxcut_kron_d10")["graph"].d == 10
    assert max(I.hypercube(10).ranks) == 2


@pytest.mark.parametrize("g", [I.grid_4x8(), I.kron_sum_products(5, 4, 2), I.complete(4)], ids=lambda g: g.name)
def test_maxcut_encoding(g):
    d = g.d
    prob = P.maxcut(g.cores)
    L = np.diag(g.dense.sum(1)) - g.dense
    vC, idx = _vectt_dense(0.25 * L, d)
    assert np.allclose(tt.full(prob["C"]), vC, atol=1e-12)
    X = np.random.default_rng(0).standard_normal((2 ** d, 2 ** d))
    vX, _ = _vectt_dense(X, d)
    # A_eq vec X keeps exactly the diagonal; K_Y keeps exactly the off-diagonal
    diag_mask, _ = _vectt_dense(np.eye(2 ** d), d)
    assert np.allclose(tt.full(tt.matvec(prob["Aeq"], [G for G in tt.tt_svd(vX, [4] * d)])), vX * diag_mask,
                       atol=1e-9)
    Kd = tt.full_mat(prob["KY"])
    assert np.allclose(np.diag(Kd), 1 - diag_mask) and np.allclose(Kd, np.diag(np.diag(Kd)))
    assert np.allclose(tt.full(prob["Beq"]), diag_mask)
    # rank statements of Sec. 4.1: rank A_eq = 1, rank K_Y = 2 (after rounding), rank C <= 2 rank A_G
    assert max(tt.ranks(prob["Aeq"])) == 1
    assert max(tt.ranks(tt.round_tt(prob["KY"], 1e-12, "rel")[0])) == 2
    assert max(tt.ranks(tt.round_tt(prob["C"], 1e-12, "rel")[0])) <= 2 * max(g.ranks)


def test_theta_encoding():
    g = I.c5_plus_3k1()
    d = g.d
    prob = P.theta(g.cores)
    n = 2 ** d
    X = np.random.default_rng(1).standard_normal((n, n))
    vX, idx = _vectt_dense(X, d)
    Aeq = tt.full_mat(prob["Aeq"])
    out = Aeq @ vX
    # slot (0,0) holds tr X; edge slots hold X_uv; everything else is idle
    assert np.isclose(out[idx[0, 0]], np.trace(X))
    for u in range(n):
        for v in range(n):
            if g.dense[u, v]:
                assert np.isclose(out[idx[u, v]], X[u, v])
            elif (u, v) != (0, 0):
                assert out[idx[u, v]] == 0
    K = np.diag(tt.full_mat(prob["KY"]))
    active = np.zeros((n, n))
    active[g.dense > 0] = 1
    active[0, 0] = 1
    assert np.allclose(K, 1 - _vectt_dense(active, d)[0])
    assert np.allclose(tt.full(prob["C"]), 1.0)
    assert np.allclose(tt.full_mat(prob["AeqT"]), Aeq.T)
    # rank statements of Sec. 4.2
    rA = max(g.ranks)
    assert max(tt.ranks(tt.round_tt(prob["Aeq"], 1e-12, "rel")[0])) <= rA + 1
    assert max(tt.ranks(tt.round_tt(prob["KY"], 1e-12, "rel")[0])) <= rA + 2


def test_cc_encoding():
    g = I.signed_kron(4, 6, 4)
    d, n = g.d, 2 ** g.d
    negdeg = np.maximum(-g.dense, 0).sum(1)
    nd_tt = tt.tt_svd(negdeg, [2] * d, tol=1e-15)
    prob = P.cc(g.cores, nd_tt)
    C = g.dense + np.diag(negdeg)
    Cp, Cm = np.maximum(g.dense, 0), np.maximum(-g.dense, 0)
    assert np.allclose(C, Cp + np.diag(Cm.sum(1)) - Cm)
    assert np.allclose(tt.full(prob["C"]), _vectt_dense(C, d)[0], atol=1e-10)
    offd = _vectt_dense(np.ones((n, n)) - np.eye(n), d)[0]
    assert np.allclose(np.diag(tt.full_mat(prob["Aineq"])), offd)
    assert np.allclose(np.diag(tt.full_mat(prob["KT"])), 1 - offd)
