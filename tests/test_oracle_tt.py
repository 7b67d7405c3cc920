"""Pins of the oracle TT library (CPU): the paper's worked vec_TT example,
frame identities, environments against explicit frames, the Hadamard and
Kronecker identities of Sec. 3.3, and rounding against TT-SVD bounds."""
import json
import os

import numpy as np
import pytest

from oracle import tt

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_tt(rng, ranks, m):
    return [rng.standard_normal((ranks[k], m, ranks[k + 1])) for k in range(len(ranks) - 1)]


def test_vec_tt_worked_example():
    g = json.load(open(os.path.join(GOLD, "vec_tt_example.json")))
    M = np.array(g["M"], dtype=float)
    # M = [[1,2],[3,4]] kron J_2 exactly: a rank-1 TT matrix with two 2x2 cores
    cores = tt.rank1_mat([np.array([[1.0, 2.0], [3.0, 4.0]]), np.ones((2, 2))])
    assert np.array_equal(tt.full_mat(cores), M)
    assert np.array_equal(M.reshape(-1), np.array(g["vec"], dtype=float))
    assert np.array_equal(tt.full(tt.vec_tt(cores)), np.array(g["vec_tt"], dtype=float))


def test_frame_identity_all_cores():
    rng = np.random.default_rng(0)
    T = _rand_tt(rng, [1, 3, 5, 4, 2, 1], 4)
    v = tt.full(T)
    for k in range(len(T)):
        F = tt.frame(T, k)
        assert np.allclose(F @ T[k].reshape(-1), v, rtol=1e-12, atol=1e-12)


def test_environments_equal_frame_projection():
    """W_{!=k}^T O W_{!=k} from cached environments == explicit frames x dense O."""
    rng = np.random.default_rng(1)
    d = 4
    W = tt.orth_left(_rand_tt(rng, [1, 3, 6, 3, 1], 4))
    O = [rng.standard_normal((r0, 4, 4, r1)) for r0, r1 in zip([1, 2, 3, 2], [2, 3, 2, 1])]
    Od = tt.full_mat(O)
    left, right = tt.envs(W, O, W)
    for k in range(d):
        F = tt.frame(W, k)
        ref = F.T @ Od @ F
        got = tt.local_dense(left[k], O[k], right[k])
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
        x = rng.standard_normal(W[k].shape)
        y = tt.local_apply(left[k], O[k], x, right[k])
        assert np.allclose(y.reshape(-1), ref @ x.reshape(-1), atol=1e-10 * np.abs(ref).max())


def test_hadamard_identity():
    """vec_TT(M o N) = diag_TT(vec_TT M) vec_TT N (Sec. 3.3 remark)."""
    rng = np.random.default_rng(2)
    M = [rng.standard_normal(s) for s in [(1, 2, 2, 3), (3, 2, 2, 2), (2, 2, 2, 1)]]
    N = [rng.standard_normal(s) for s in [(1, 2, 2, 2), (2, 2, 2, 2), (2, 2, 2, 1)]]
    lhs = tt.full(tt.vec_tt(M))
    had = tt.full_mat(M) * tt.full_mat(N)
    rhs = tt.full(tt.matvec(tt.diag_tt(tt.vec_tt(M)), tt.vec_tt(N)))
    # compare through vec_TT of the dense Hadamard product
    got = tt.full(tt.tt_svd(_vectt_dense(had, 3), [4] * 3))
    assert np.allclose(rhs, _vectt_dense(had, 3), atol=1e-12)
    assert np.allclose(got, rhs, atol=1e-10)
    assert lhs.shape == rhs.shape


def _vectt_dense(A, d):
    """vec_TT ordering of a dense 2^d x 2^d matrix by explicit index interleaving."""
    n = 2 ** d
    out = np.zeros(n * n)
    for r in range(n):
        for c in range(n):
            idx = 0
            for k in range(d):
                a = (r >> (d - 1 - k)) & 1
                b = (c >> (d - 1 - k)) & 1
                idx = idx * 4 + 2 * a + b
            out[idx] = A[r, c]
    return out


def test_kronecker_action():
    """(A kron_TT B) vec_TT(X) = vec_TT(A X B^T) with per-core Kronecker products."""
    rng = np.random.default_rng(3)
    d = 3
    A = [rng.standard_normal(s) for s in [(1, 2, 2, 2), (2, 2, 2, 3), (3, 2, 2, 1)]]
    B = [rng.standard_normal(s) for s in [(1, 2, 2, 3), (3, 2, 2, 2), (2, 2, 2, 1)]]
    X = [rng.standard_normal(s) for s in [(1, 2, 2, 2), (2, 2, 2, 2), (2, 2, 2, 1)]]
    lhs = tt.full(tt.matvec(tt.kron(A, B), tt.vec_tt(X)))
    Ad, Bd, Xd = tt.full_mat(A), tt.full_mat(B), tt.full_mat(X)
    assert np.allclose(lhs, _vectt_dense(Ad @ Xd @ Bd.T, d), atol=1e-10)


def test_vec_tt_of_dense_matches_interleaving():
    rng = np.random.default_rng(4)
    X = [rng.standard_normal(s) for s in [(1, 2, 2, 2), (2, 2, 2, 3), (3, 2, 2, 1)]]
    assert np.allclose(tt.full(tt.vec_tt(X)), _vectt_dense(tt.full_mat(X), 3), atol=1e-12)


@pytest.mark.parametrize("ranks", [[1, 4, 7, 4, 1], [1, 2, 8, 8, 8, 2, 1]])
def test_round_exact_recovery(ranks):
    rng = np.random.default_rng(5)
    T = _rand_tt(rng, ranks, 4)
    T2 = tt.add([T, T], [1.0, 1.0])
    R, zeta = tt.round_tt(T2, 1e-12, "rel")
    assert max(tt.ranks(R)) <= max(ranks)
    assert np.linalg.norm(tt.full(R) - 2 * tt.full(T)) <= 1e-11 * np.linalg.norm(tt.full(T))
    assert zeta <= 1e-11 * np.linalg.norm(tt.full(T))


@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-6])
def test_round_error_bound_and_zeta(tol):
    """||T - round(T)||_F <= eps, zeta equals the true error, and each bond's
    rank is no larger than that of the TT-SVD of the dense tensor at eps/sqrt(d-1)."""
    rng = np.random.default_rng(6)
    T = _rand_tt(rng, [1, 4, 16, 16, 4, 1], 4)
    for k in range(len(T)):
        T[k] = T[k] * np.geomspace(1, 1e-4, T[k].shape[-1])[None, None, :]
    eps = tol * tt.norm(T)
    R, zeta = tt.round_tt(T, eps, "abs")
    err = np.linalg.norm(tt.full(R) - tt.full(T))
    assert err <= eps * (1 + 1e-10)
    assert abs(err - zeta) <= 1e-9 * tt.norm(T)
    ref = tt.tt_svd(tt.full(T), [4] * len(T), tol=eps / tt.norm(T))
    assert all(a <= b for a, b in zip(tt.ranks(R), tt.ranks(ref)))


def test_dot_norm_sandwich_dense():
    rng = np.random.default_rng(7)
    x = _rand_tt(rng, [1, 3, 4, 2, 1], 4)
    y = _rand_tt(rng, [1, 2, 5, 3, 1], 4)
    A = [rng.standard_normal(s) for s in [(1, 4, 4, 2), (2, 4, 4, 2), (2, 4, 4, 3), (3, 4, 4, 1)]]
    assert np.isclose(tt.dot(x, y), tt.full(x) @ tt.full(y), rtol=1e-12)
    assert np.isclose(tt.norm(x), np.linalg.norm(tt.full(x)), rtol=1e-12)
    assert np.isclose(tt.sandwich(x, A, y), tt.full(x) @ tt.full_mat(A) @ tt.full(y), rtol=1e-10)


def test_degenerate_projector_example():
    """Sec. 2.3 example: A = [[0,1],[1,0]], frame [0,1]^T gives a singular (zero) projection."""
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    F = np.array([[0.0], [1.0]])
    assert np.linalg.det(A) != 0
    assert (F.T @ A @ F)[0, 0] == 0.0
