"""Rank floor of the n = 2^10 Kronecker MaxCut optimum (CPU, oracle only).

The dense HKM oracle's optimal X* of the C2 instance (sum of 4 Kronecker
products of 10 random symmetric 2 x 2 factors, seed 2) has matrix rank 2, but
its vec_TT ranks are high.  Truncating vec_TT(X*) with the quasi-optimal TT-SVD
(Sec. 2.3; Oseledets 2011: within sqrt(d-1) of the best rank-r error) to the
iterate caps that a TT interior-point method would use shows the floor that
the cap puts under primal feasibility: at rank 32 the unit-diagonal residual
||diag X~ - 1|| / (1 + ||1||) stays above 1e-3, at rank 64 above 2e-4 (the
stopping threshold eps_p of Sec. 5.1 at eps_gap = 1e-4), and every truncation
leaves X~ indefinite, so a positive-definite iterate near X* needs a spectral
shift of that size on the diagonal (Cor. 1), which moves diag X by the same
amount.  The dual slack Z* needs TT rank <= 32 (exact to 1e-7).
"""
import numpy as np
import pytest

import instances as I
from oracle import certificate as cert, problems as OP, sdp_dense as S, tt


@pytest.fixture(scope="module")
def c2_optimum():
    g = I.kron_sum_products(10, 4, 2)
    res = S.solve(OP.maxcut_dense(g.dense), tol_gap=1e-10, tol_feas=1e-10)
    return res


def _vec(M, d):
    idx = cert.vec_index(d)
    v = np.zeros(4 ** d)
    v[idx.ravel()] = M.ravel()
    return v


def _truncate(M, d, r):
    cores = tt.tt_svd(_vec(M, d), [4] * d, tol=1e-15, max_rank=r)
    return cert.dense_matrix(cores)


def test_c2_optimum_has_matrix_rank_two(c2_optimum):
    X = 0.5 * (c2_optimum["X"] + c2_optimum["X"].T)
    ev = np.linalg.eigvalsh(X)[::-1]
    assert ev[1] > 10.0 and ev[2] < 1e-3 * ev[0]


@pytest.mark.parametrize("rank,eps_p_min", [(32, 1e-3), (64, 2e-4)])
def test_c2_primal_floor_at_iterate_cap(c2_optimum, rank, eps_p_min):
    d, n = 10, 1024
    X = 0.5 * (c2_optimum["X"] + c2_optimum["X"].T)
    Xt = _truncate(X, d, rank)
    eps_p = np.linalg.norm(np.diag(Xt) - 1.0) / (1.0 + np.sqrt(n))
    lam = np.linalg.eigvalsh(0.5 * (Xt + Xt.T))[0]
    assert eps_p > eps_p_min
    assert lam < -1e-2          # indefinite: a PD iterate needs a shift of at least |lam| on the diagonal


def test_c2_dual_slack_is_low_rank(c2_optimum):
    Z = 0.5 * (c2_optimum["Z"] + c2_optimum["Z"].T)
    Zt = _truncate(Z, 10, 32)
    assert np.linalg.norm(Zt - Z) <= 1e-6 * np.linalg.norm(Z)
