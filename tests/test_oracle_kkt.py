"""Pins of the dense Newton-system oracle (oracle/kkt.py) — CPU only.

The dense Newton solve is the reference of the GPU Newton-step parity tests, so
it is pinned here against what the mathematics fixes, independently of its own
code:

* The matrix-form Newton equations.  The solution of eq. (tt-kkt-newton-system)
  in the padded vec_TT space, mapped back to n x n matrices with an index map
  written here from the vec_TT definition (Def. "TT Vectorisation", pinned by the
  worked example in tests/golden/vec_tt_example.json), must satisfy the
  linearised optimality conditions of the SDP and its dual (Sec. 2.2, Defs.
  "SDP" and "The Dual SDP"), written out here from the dense problem data of
  each encoding (Sec. 4):
    - primal rows: A(X + dX) = b on the active constraints, dY = 0 on idle ones;
    - dual row: Z + dZ + C - A^T(Y + dY) (+/- inequality multipliers) = 0;
    - complementarity: Z dX + dX Z + X dZ + dZ X = 2 sigma mu I - (ZX + XZ)
      (AHO), Z dX + dZ X = sigma mu I - ZX (XZ), and for the inequalities
      T o dX + X o dT = sigma mu - T o X on the active pairs.
  Catches a transposed Kronecker factor (XZ operators), a sign on A_eq^T or on
  the inequality term, a wrong R_c coefficient (mu vs 2 mu), a dropped K_Y
  mask and a wrong slack orientation.
* Eq. (reduced_kkt_system) with the full frame W = I gives the unreduced
  solution (catches a sign or missing L_X R_d term in the reduced right-hand
  side, or a projection of the product L_X A_eq^T in place of the chain).
* The Sec. 3.3 block elimination equals an LU solve of the reduced system on
  random orthonormal frames W (N x p, p < N) (catches a wrong Schur complement
  or elimination order).
* Lemma "AMEn Directions as Inexact Newton Directions": with R~ within a
  relative delta_R of R, K~ within the lemma's relative tolerance of K and a
  direction meeting the rounded forcing condition, the exact forcing condition
  ||K dU + R|| <= eta ||R|| holds (checked densely up to d = 5).
* Planted mistakes: each of the errors above, planted in a copy of the oracle's
  operators, makes the matrix-form check fail.
"""
import numpy as np
import pytest

import instances as I
from oracle import kkt, problems as OP, tt


# --------------------------------------------------------------------------
# helpers written from the definitions (not from the oracle's code)
# --------------------------------------------------------------------------

def vec_index(d):
    """idx[r, c] = vec_TT position of entry (r, c): mode k holds the digit
    2 * (bit k of r) + (bit k of c), core 0 the most significant bits."""
    n = 2 ** d
    idx = np.zeros((n, n), dtype=np.int64)
    for r in range(n):
        for c in range(n):
            v = 0
            for k in range(d):
                v = 4 * v + 2 * ((r >> (d - 1 - k)) & 1) + ((c >> (d - 1 - k)) & 1)
            idx[r, c] = v
    return idx


def to_vec(M, idx):
    v = np.zeros(M.size)
    v[idx.reshape(-1)] = M.reshape(-1)
    return v


def to_tt(M, idx, d):
    return tt.tt_svd(to_vec(M, idx), [4] * d, tol=1e-15)


def spd(rng, n, shift=1.0):
    G = rng.standard_normal((n, n))
    return G @ G.T / n + shift * np.eye(n)


def offdiag(M):
    return M - np.diag(np.diag(M))


def _state(kind, rng, d, graph):
    """Random strictly interior iterate (dense matrices) for an encoding."""
    n = 2 ** d
    X, Z = spd(rng, n), spd(rng, n)
    Y = rng.standard_normal((n, n))
    T = None
    if kind == "cc":
        T = np.abs(rng.standard_normal((n, n))) + 0.1
        T = offdiag(0.5 * (T + T.T))
        # X strictly feasible for X_uv >= 0 off the diagonal
        X = spd(rng, n) + 0.5 * np.ones((n, n))
    return X, Y, Z, T


def _problem(kind, graph):
    d = graph.d
    if kind == "maxcut":
        return OP.maxcut(graph.cores)
    if kind == "theta":
        return OP.theta(graph.cores)
    negdeg = np.maximum(-graph.dense, 0).sum(1)
    return OP.cc(graph.cores, tt.tt_svd(negdeg, [2] * d, tol=1e-15))


def _matrix_form_residuals(kind, A, X, Y, Z, T, dX, dY, dZ, dT, sm, direction):
    """Largest violations of the linearised optimality conditions (dense)."""
    n = X.shape[0]
    I_n = np.eye(n)
    out = {}
    if kind == "maxcut":
        C = 0.25 * (np.diag(A.sum(1)) - A)
        out["primal"] = np.abs(np.diag(X + dX) - 1.0).max()
        out["idle"] = np.abs(offdiag(dY)).max()
        out["dual"] = np.abs(Z + dZ + C - np.diag(np.diag(Y + dY))).max()
    elif kind == "theta":
        C = np.ones((n, n))
        E = A > 0.5
        Yn = Y + dY
        out["primal"] = max(np.abs((X + dX)[E]).max(), abs(np.trace(X + dX) - 1.0))
        idle = ~E
        idle[0, 0] = False
        out["idle"] = np.abs(dY[idle]).max()
        out["dual"] = np.abs(Z + dZ + C - np.where(E, Yn, 0.0) - Yn[0, 0] * I_n).max()
    else:  # cc, >= convention: X_uv >= 0 off the diagonal, multipliers T >= 0
        Cm = np.maximum(-A, 0.0)
        C = A + np.diag(Cm.sum(1))
        out["primal"] = np.abs(np.diag(X + dX) - 1.0).max()
        out["idle"] = np.abs(offdiag(dY)).max()
        out["dual"] = np.abs(Z + dZ + C - np.diag(np.diag(Y + dY)) + offdiag(T + dT)).max()
        comp_t = T * dX + X * dT - (sm - T * X)
        out["comp_t"] = np.abs(offdiag(comp_t)).max()
        out["idle_t"] = np.abs(np.diag(dT)).max()
    if direction == "aho":
        lhs = Z @ dX + dX @ Z + X @ dZ + dZ @ X
        rhs = 2.0 * sm * I_n - (Z @ X + X @ Z)
    else:
        lhs = Z @ dX + dZ @ X
        rhs = sm * I_n - Z @ X
    out["comp"] = np.abs(lhs - rhs).max()
    return out


def _solve_matrix_form(kind, graph, direction, seed, ops=None):
    d = graph.d
    idx = vec_index(d)
    rng = np.random.default_rng(seed)
    prob = _problem(kind, graph)
    X, Y, Z, T = _state(kind, rng, d, graph)
    mu = float(rng.uniform(0.1, 1.0))
    sm = float(rng.uniform(0.0, 0.5)) * mu     # the corrector's centring target sigma mu
    Xt, Yt, Zt = to_tt(X, idx, d), to_tt(Y, idx, d), to_tt(Z, idx, d)
    Tt = to_tt(T, idx, d) if T is not None else None
    dx, dy, dt, dz = kkt.newton_dense(prob, Xt, Yt, Zt, Tt, mu, direction, sigma_mu=sm)
    M = lambda v: v[idx]
    dT = M(dt) if dt is not None else None
    res = _matrix_form_residuals(kind, graph.dense, X, Y, Z, T, M(dx), M(dy), M(dz), dT, sm, direction)
    scale = 1.0 + max(np.abs(X).max(), np.abs(Z).max(), np.abs(Y).max())
    return res, scale


GRAPHS = {
    "maxcut": lambda: I.kron_sum_products(3, 2, 11),
    "theta": lambda: I.c5_plus_3k1(),
    "cc": lambda: I.signed_kron(3, 2, 7),
}


@pytest.mark.parametrize("direction", ["aho", "xz"])
@pytest.mark.parametrize("kind", ["maxcut", "theta", "cc"])
def test_newton_dense_satisfies_matrix_form_equations(kind, direction):
    if kind == "cc" and direction == "xz":
        pytest.skip("the XZ warm-up is not used with inequality constraints")
    res, scale = _solve_matrix_form(kind, GRAPHS[kind](), direction, seed=3)
    for name, v in res.items():
        assert v <= 1e-10 * scale, f"{kind}/{direction}: {name} violated by {v:.3e}"


def test_newton_dense_matrix_form_d4_maxcut():
    # a second size (4 x 4 grid of blocks: n = 16, N = 256 per block)
    res, scale = _solve_matrix_form("maxcut", I.kron_sum_products(4, 3, 5), "aho", seed=9)
    for name, v in res.items():
        assert v <= 1e-10 * scale, f"{name} violated by {v:.3e}"


# --------------------------------------------------------------------------
# planted mistakes: each one must break the matrix-form check
# --------------------------------------------------------------------------

def _plant(monkeypatch, which):
    orig_L, orig_res = kkt.L_ops, kkt.residuals_dense

    if which == "kron_transposed":
        def L_bad(X, Z, direction):
            LZ, LX = orig_L(X, Z, direction)
            d = len(X)
            Id = kkt.identity_mat_tt(d)
            if direction == "xz":      # Z x I -> I x Z
                LZ = tt.kron(Id, tt.unvec_tt(Z))
            return LZ, LX
        monkeypatch.setattr(kkt, "L_ops", L_bad)
    elif which == "rc_coefficient":
        def res_bad(prob, X, Y, Z, T, mu, direction, sigma_mu=None):
            Rd, Rp, Rt, Rc = orig_res(prob, X, Y, Z, T, mu, direction, sigma_mu)
            target = mu if sigma_mu is None else sigma_mu
            Ivec = tt.full(tt.rank1_vec([np.array([1.0, 0, 0, 1])] * prob["d"]))
            return Rd, Rp, Rt, Rc + target * Ivec          # 2 mu I -> mu I
        monkeypatch.setattr(kkt, "residuals_dense", res_bad)
    elif which == "aeqT_sign":
        def res_bad(prob, X, Y, Z, T, mu, direction, sigma_mu=None):
            Rd, Rp, Rt, Rc = orig_res(prob, X, Y, Z, T, mu, direction, sigma_mu)
            AeqT = tt.full_mat(prob["AeqT"])
            return Rd + 2.0 * AeqT @ tt.full(Y), Rp, Rt, Rc   # - Aeq^T Y -> + Aeq^T Y
        monkeypatch.setattr(kkt, "residuals_dense", res_bad)
    elif which == "ineq_sign":
        def res_bad(prob, X, Y, Z, T, mu, direction, sigma_mu=None):
            Rd, Rp, Rt, Rc = orig_res(prob, X, Y, Z, T, mu, direction, sigma_mu)
            AiT = tt.full_mat(prob["AineqT"])
            return Rd + 2.0 * prob["sense"] * (AiT @ tt.full(T)), Rp, Rt, Rc
        monkeypatch.setattr(kkt, "residuals_dense", res_bad)
    else:
        raise ValueError(which)


@pytest.mark.parametrize("which,kind,direction", [
    ("kron_transposed", "maxcut", "xz"),
    ("rc_coefficient", "maxcut", "aho"),
    ("aeqT_sign", "theta", "aho"),
    ("ineq_sign", "cc", "aho"),
])
def test_planted_mistakes_are_caught(monkeypatch, which, kind, direction):
    _plant(monkeypatch, which)
    res, scale = _solve_matrix_form(kind, GRAPHS[kind](), direction, seed=3)
    worst = max(res.values())
    assert worst > 1e-6 * scale, f"planted mistake {which} went unnoticed ({res})"


# --------------------------------------------------------------------------
# reduced system and block elimination (Sec. 3.3)
# --------------------------------------------------------------------------

def _blocks(kind, graph, direction, seed):
    d = graph.d
    idx = vec_index(d)
    rng = np.random.default_rng(seed)
    prob = _problem(kind, graph)
    X, Y, Z, T = _state(kind, rng, d, graph)
    mu = float(rng.uniform(0.1, 1.0))
    Xt, Yt, Zt = to_tt(X, idx, d), to_tt(Y, idx, d), to_tt(Z, idx, d)
    Tt = to_tt(T, idx, d) if T is not None else None
    return prob, (Xt, Yt, Zt, Tt, mu), kkt.system_blocks(prob, Xt, Yt, Zt, Tt, mu, direction, sigma_mu=0.3 * mu)


@pytest.mark.parametrize("kind", ["maxcut", "theta", "cc"])
def test_reduced_system_full_frame_equals_unreduced(kind):
    direction = "aho"
    prob, st, B = _blocks(kind, GRAPHS[kind](), direction, seed=5)
    Xt, Yt, Zt, Tt, mu = st
    full = kkt.newton_dense(prob, Xt, Yt, Zt, Tt, mu, direction, sigma_mu=0.3 * mu)
    N = B["Aeq"].shape[0]
    W = np.eye(N)
    K, rhs = kkt.reduced_system(B, W)
    sol = np.linalg.solve(K, rhs)
    parts = np.split(sol, 3 if B["ineq"] else 2)
    dX, dY = parts[0], parts[1]
    dT = parts[2] if B["ineq"] else None
    dZ = kkt.dz_local(B, W, dY, dT)
    ref = [full[0], full[1], full[3]] + ([full[2]] if B["ineq"] else [])
    got = [dX, dY, dZ] + ([dT] if B["ineq"] else [])
    for a, b in zip(got, ref):
        assert np.linalg.norm(a - b) <= 1e-10 * (1 + np.linalg.norm(b))


@pytest.mark.parametrize("kind", ["maxcut", "theta", "cc"])
@pytest.mark.parametrize("p", [12, 40])
def test_block_elimination_equals_lu_of_reduced_system(kind, p):
    direction = "aho"
    _, _, B = _blocks(kind, GRAPHS[kind](), direction, seed=8)
    N = B["Aeq"].shape[0]
    rng = np.random.default_rng(p)
    W, _ = np.linalg.qr(rng.standard_normal((N, p)))
    K, rhs = kkt.reduced_system(B, W)
    sol = np.linalg.solve(K, rhs)
    parts = np.split(sol, 3 if B["ineq"] else 2)
    dX, dY, dT, dZ = kkt.block_elimination(B, W)
    assert np.linalg.norm(dX - parts[0]) <= 1e-9 * (1 + np.linalg.norm(parts[0]))
    assert np.linalg.norm(dY - parts[1]) <= 1e-9 * (1 + np.linalg.norm(parts[1]))
    if B["ineq"]:
        assert np.linalg.norm(dT - parts[2]) <= 1e-9 * (1 + np.linalg.norm(parts[2]))
    dz_ref = kkt.dz_local(B, W, parts[1], parts[2] if B["ineq"] else None)
    assert np.linalg.norm(dZ - dz_ref) <= 1e-9 * (1 + np.linalg.norm(dz_ref))


def test_reduced_system_is_not_projection_of_product():
    # The chained block (W^T L_X W)(W^T Aeq^T W) differs from W^T L_X Aeq^T W
    # for a proper frame; the oracle must keep the chain (Sec. 3.3).
    _, _, B = _blocks("maxcut", GRAPHS["maxcut"](), "aho", seed=2)
    N = B["Aeq"].shape[0]
    W, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((N, 20)))
    K, _ = kkt.reduced_system(B, W)
    chain = K[20:, 20:]
    proj_prod = W.T @ B["LX"] @ B["AeqT"] @ W
    assert np.allclose(chain, (W.T @ B["LX"] @ W) @ (W.T @ B["AeqT"] @ W))
    assert not np.allclose(chain, proj_prod, atol=1e-6)


# --------------------------------------------------------------------------
# Lemma: AMEn directions as inexact Newton directions (forcing condition)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,graph", [
    ("maxcut", lambda: I.kron_sum_products(3, 2, 11)),
    ("maxcut", lambda: I.kron_sum_products(5, 2, 3)),
    ("cc", lambda: I.signed_kron(3, 2, 7)),
], ids=["maxcut_d3", "maxcut_d5", "cc_d3"])
def test_lemma_forcing_condition_dense(kind, graph):
    g = graph()
    _, _, B = _blocks(kind, g, "aho", seed=4)
    K, mR = kkt.assemble(B)
    R = -mR
    nR = np.linalg.norm(R)
    kF = np.linalg.norm(K) * np.linalg.norm(np.linalg.inv(K))
    rng = np.random.default_rng(17)
    for eta, delta_R, eta_t in [(0.5, 0.05, 0.2), (0.1, 0.01, 0.05), (0.9, 0.2, 0.4)]:
        assert delta_R + (1 + delta_R) * eta_t <= eta < 1
        delta_K = (eta - delta_R - (1 + delta_R) * eta_t) / ((1 + delta_R) * (1 + eta_t))
        # R~ within relative delta_R of R
        e = rng.standard_normal(R.shape)
        Rt = R + delta_R * nR * e / np.linalg.norm(e)
        # K~ within the lemma's relative tolerance delta_K / ((1 + delta_K) kappa_F(K))
        E = rng.standard_normal(K.shape)
        Kt = K + (delta_K / ((1 + delta_K) * kF)) * np.linalg.norm(K) * E / np.linalg.norm(E)
        # a direction meeting the rounded forcing condition with equality
        gvec = rng.standard_normal(R.shape)
        gvec *= eta_t * np.linalg.norm(Rt) / np.linalg.norm(gvec)
        dU = np.linalg.solve(Kt, -Rt + gvec)
        assert np.linalg.norm(Kt @ dU + Rt) <= eta_t * np.linalg.norm(Rt) * (1 + 1e-9)
        assert np.linalg.norm(K @ dU + R) <= eta * nR
