"""Pins of the certificate evaluator (oracle/certificate.py) — CPU only.

* Validity: lb <= p* <= ub for the optimum of the dense oracle and for randomly
  perturbed iterates, on instances whose p* is a closed form (K_n: n^2/4, the
  4x8 grid: 52, theta(C5 u 3K1) = 3 + sqrt 5, theta(Q_4) = 8) or the dense
  oracle's value (Kronecker MaxCut, signed correlation clustering).  A wrong
  sign in a bound or a missed trace factor breaks one side.
* Tightness: at the dense optimum the width (ub - lb)/(1 + |ub|) is <= 1e-6.
* Repair: the repaired primal matrix is feasible (unit diagonal and PSD,
  nonnegative pairs for CC, zero edges and unit trace for theta).
* vec_TT: dense_matrix of the TT-SVD of a matrix's vec_TT vector returns the
  matrix (index map of Def. "TT Vectorisation").
"""
import math

import numpy as np
import pytest

import instances as I
from oracle import certificate as Ce, problems as P, sdp_dense as S, tt


def _padded(kind, A, r):
    """Multipliers of the dense oracle in the padded TT layout (Y, T)."""
    n = A.shape[0]
    if kind == "maxcut":
        return np.diag(r["y"]), None
    if kind == "theta":
        Y = np.zeros((n, n))
        Y[0, 0] = r["y"][0]
        iu, ju = np.nonzero(np.triu(A, 1))
        Y[iu, ju] = r["y"][1:] / 2
        Y[ju, iu] = r["y"][1:] / 2
        return Y, None
    iu, ju = np.triu_indices(n, 1)
    T = np.zeros((n, n))
    T[iu, ju] = r["t"] / 2
    T = T + T.T
    return np.diag(r["y"]), T


CASES = [
    ("maxcut", lambda: I.complete(3).dense, 16.0),
    ("maxcut", lambda: I.grid_4x8().dense, 52.0),
    ("maxcut", lambda: I.kron_sum_products(4, 3, 5).dense, None),
    ("theta", lambda: I.c5_plus_3k1().dense, 3 + math.sqrt(5)),
    ("theta", lambda: I.hypercube(4).dense, 8.0),
    ("cc", lambda: I.signed_kron(3, 2, 7).dense, None),
    ("cc", lambda: I.signed_kron(4, 3, 1).dense, None),
]
IDS = ["K8", "grid", "kron_d4", "C5+3K1", "Q4", "cc_d3", "cc_d4"]


def _dense(kind, A):
    return {"maxcut": P.maxcut_dense, "theta": P.theta_dense, "cc": P.cc_dense}[kind](A)


@pytest.mark.parametrize("kind,graph,value", CASES, ids=IDS)
def test_certificate_valid_and_tight(kind, graph, value):
    A = graph()
    r = S.solve(_dense(kind, A))
    pstar = value if value is not None else 0.5 * (r["pobj"] + r["dobj"])
    Y, T = _padded(kind, A, r)
    c = Ce.certificate(kind, A, r["X"], Y, r["Z"], T)
    tol = 1e-7 * (1 + abs(pstar))
    assert c["lb"] <= pstar + tol and pstar <= c["ub"] + tol
    assert c["width"] <= 1e-6
    rng = np.random.default_rng(3)
    n = A.shape[0]
    for scale in (1e-3, 1e-1):
        E = rng.standard_normal((n, n)) * scale
        Ey = rng.standard_normal((n, n)) * scale
        Et = np.abs(rng.standard_normal((n, n))) * scale if T is not None else None
        Xp, Yp = r["X"] + E + E.T, Y + Ey + Ey.T
        Tp = T + Et + Et.T if T is not None else None
        cp = Ce.certificate(kind, A, Xp, Yp, r["Z"], Tp)
        assert cp["lb"] <= pstar + tol, (scale, cp)
        assert pstar <= cp["ub"] + tol, (scale, cp)


@pytest.mark.parametrize("kind,graph", [(k, g) for k, g, _ in CASES], ids=IDS)
def test_repaired_primal_is_feasible(kind, graph):
    A = graph()
    n = A.shape[0]
    rng = np.random.default_rng(11)
    X = rng.standard_normal((n, n))
    Xr, _ = Ce.repaired_primal(kind, A, X + X.T)
    assert np.allclose(Xr, Xr.T)
    assert np.linalg.eigvalsh(Xr)[0] >= -1e-10
    if kind in ("maxcut", "cc"):
        assert np.allclose(np.diag(Xr), 1.0)
    if kind == "cc":
        assert (Xr - np.diag(np.diag(Xr))).min() >= -1e-12
    if kind == "theta":
        assert abs(np.trace(Xr) - 1.0) < 1e-12
        assert np.abs(Xr[A > 0.5]).max() == 0.0


def test_dense_matrix_roundtrip():
    d = 4
    n = 2 ** d
    M = np.random.default_rng(5).standard_normal((n, n))
    v = np.zeros(n * n)
    v[Ce.vec_index(d).reshape(-1)] = M.reshape(-1)
    cores = tt.tt_svd(v, [4] * d, tol=1e-15)
    assert np.allclose(Ce.dense_matrix(cores), M, atol=1e-12)
