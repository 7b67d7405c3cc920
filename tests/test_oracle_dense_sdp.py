"""Pins of the dense IPM oracle against closed-form SDP values (CPU)."""
import json
import math
import os

import numpy as np
import pytest

import instances as I
from oracle import problems as P, sdp_dense as S


def _rel(a, b):
    return abs(a - b) / (1 + abs(b))


@pytest.mark.parametrize("d", [3, 4, 5])
def test_maxcut_complete(d):
    n = 2 ** d
    r = S.solve(P.maxcut_dense(I.complete(d).dense))
    assert r["status"] == "optimal" and _rel(r["pobj"], n * n / 4) < 1e-8


@pytest.mark.parametrize("d", [3, 4, 5])
def test_maxcut_odd_cycle(d):
    g = I.odd_cycle_plus_isolated(d)
    m = 2 ** d - 1
    r = S.solve(P.maxcut_dense(g.dense))
    assert _rel(r["pobj"], m / 2 * (1 + math.cos(math.pi / m))) < 1e-8


def test_maxcut_bipartite_grid_and_hypercube():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
    r = S.solve(P.maxcut_dense(I.grid_4x8().dense))
    assert _rel(r["pobj"], gold["grid_4x8_maxcut"]) < 1e-8
    # unique optimum X* = x x^T with the checkerboard x (Sec. 4.1 reading)
    x = np.array([(-1) ** (i + j) for i in range(4) for j in range(8)], dtype=float)
    assert np.linalg.norm(r["X"] - np.outer(x, x)) < 1e-3
    r = S.solve(P.maxcut_dense(I.hypercube(5).dense))
    assert _rel(r["pobj"], 5 * 16) < 1e-8


@pytest.mark.parametrize("d", [3, 4, 5])
def test_theta_hypercube(d):
    r = S.solve(P.theta_dense(I.hypercube(d).dense))
    assert _rel(r["pobj"], 2 ** (d - 1)) < 1e-8


def test_theta_c5_plus_isolated():
    r = S.solve(P.theta_dense(I.c5_plus_3k1().dense))
    assert _rel(r["pobj"], 3 + math.sqrt(5)) < 1e-8


def test_cc_closed_forms():
    rng = np.random.default_rng(0)
    n = 8
    W = rng.uniform(size=(n, n)); W = 0.5 * (W + W.T); np.fill_diagonal(W, 0)
    r = S.solve(P.cc_dense(W))
    assert _rel(r["pobj"], W.sum()) < 1e-7
    Wn = -(np.ones((n, n)) - np.eye(n))
    r = S.solve(P.cc_dense(Wn))
    assert _rel(r["pobj"], n * (n - 1)) < 1e-7


def test_certificates_weak_duality():
    """Returned iterates are feasible to 1e-9 and the dual bound is rigorous:
    Z = A^T y - C psd up to 1e-9 and b^T y >= C . X."""
    g = I.kron_sum_products(5, 4, 2)
    r = S.solve(P.maxcut_dense(g.dense))
    L = np.diag(g.dense.sum(1)) - g.dense
    C = 0.25 * L
    Z = np.diag(r["y"]) - C
    assert np.linalg.eigvalsh(Z)[0] > -1e-8
    assert np.abs(np.diag(r["X"]) - 1).max() < 1e-9
    assert np.linalg.eigvalsh(r["X"])[0] > -1e-8
    assert r["y"].sum() >= np.sum(C * r["X"]) - 1e-7


def test_step_length_theorem1():
    """Thm. 1 step vs bisection on lambda_min(M + a dM)."""
    rng = np.random.default_rng(3)
    n = 12
    B = rng.standard_normal((n, n)); M = B @ B.T + 0.1 * np.eye(n)
    dM = rng.standard_normal((n, n)); dM = dM + dM.T
    a = S.max_step(M, dM)
    lo, hi = 0.0, 100.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.linalg.eigvalsh(M + mid * dM)[0] >= 0:
            lo = mid
        else:
            hi = mid
    assert abs(a - lo) < 1e-9 * max(1, lo)
    assert S.max_step(M, np.eye(n)) == np.inf
