"""Certificate evaluator for TT iterates (oracle; test only).

For configurations whose dense interior-point solve is out of reach (the
correlation-clustering SDP at n = 4096 has about n^2/2 inequality
multipliers), the TT-IPM result is judged by a certificate computed from its
iterates: the TT cores are densified (n <= 4096), and

  * an upper bound on the SDP value p* follows from the dual iterate alone, by
    weak duality (Sec. 2.2, Def. "The Dual SDP"; Example "Maximum Cut",
    "Maximum Stable Set", "Correlation Clustering"): the dual slack implied by
    the multipliers is rebuilt from y (not taken from the Z iterate), and its
    most negative eigenvalue is charged against the trace of a feasible X,
    which is fixed by the constraints:
      MaxCut:  p* <= sum(y) - n min(0, lambda_min(Diag y - C))        (tr X = n)
      theta:   p* <= y_tr  - min(0, lambda_min(y_tr I + A o Y - J))   (tr X = 1)
      CC:      p* <= sum(y) - n min(0, lambda_min(Diag y - C - V+))   (tr X = n,
               V+ = the nonnegative part of the pair multipliers, X_uv >= 0)
  * a lower bound is the objective of a feasible X repaired from the primal
    iterate: its projection on the PSD cone scaled to unit diagonal (MaxCut),
    that matrix mixed with J until every pair entry is >= 0 (CC), or the
    iterate with its edge entries zeroed, shifted to PSD and scaled to unit
    trace (theta).

So lb <= p* <= ub holds for any iterate, and ub - lb measures how well the
iterate pair solves the SDP.  Matrices are symmetrised, (M + M^T)/2, before
use.  The padded multiplier layout is that of the TT encodings (Sec. 4): for
MaxCut and CC y = diag(Y); for theta y_tr = Y[0, 0] and the edge multipliers
are the entries of Y on the edges; for CC the pair multipliers are the
off-diagonal entries of T.
"""
from __future__ import annotations

import numpy as np

from . import tt


def vec_index(d):
    """vec_TT position of every entry (r, c) of a 2^d x 2^d matrix: the digit of
    mode k is 2 * (bit k of r) + (bit k of c), core 0 the most significant."""
    n = 2 ** d
    r = np.arange(n)[:, None]
    c = np.arange(n)[None, :]
    v = np.zeros((n, n), dtype=np.int64)
    for k in range(d):
        sh = d - 1 - k
        v = 4 * v + 2 * ((r >> sh) & 1) + ((c >> sh) & 1)
    return v


def dense_matrix(cores):
    """n x n matrix of a vec_TT vector given by its TT cores [r, 4, r']."""
    d = len(cores)
    return tt.full(cores)[vec_index(d)]


def _sym(M):
    return 0.5 * (M + M.T)


def objective_matrix(kind, A):
    """C of the dense SDP for the graph matrix A (Sec. 2.2 examples, Sec. 4)."""
    n = A.shape[0]
    if kind == "maxcut":
        return 0.25 * (np.diag(A.sum(1)) - A)
    if kind == "theta":
        return np.ones((n, n))
    if kind == "cc":
        return A + np.diag(np.maximum(-A, 0.0).sum(1))
    raise ValueError(kind)


def _lmin(M):
    return float(np.linalg.eigvalsh(_sym(M))[0])


def _psd_part(M):
    w, V = np.linalg.eigh(_sym(M))
    return (V * np.maximum(w, 0.0)) @ V.T


def _unit_diag(M):
    dg = np.diag(M).copy()
    dg[dg <= 0] = 1.0   # an all-zero row/column: its entries are 0; unit diagonal added below
    s = 1.0 / np.sqrt(dg)
    out = M * s[:, None] * s[None, :]
    np.fill_diagonal(out, 1.0)
    return out


def upper_bound(kind, A, Y, T=None):
    """Weak-duality bound on p* from the multipliers (see the module text)."""
    n = A.shape[0]
    C = objective_matrix(kind, A)
    Y = _sym(Y)
    if kind == "maxcut":
        y = np.diag(Y)
        return float(y.sum() - n * min(0.0, _lmin(np.diag(y) - C)))
    if kind == "theta":
        E = A > 0.5
        ytr = float(Y[0, 0])
        Zr = ytr * np.eye(n) + np.where(E, Y, 0.0) - C
        return float(ytr - min(0.0, _lmin(Zr)))
    if kind == "cc":
        y = np.diag(Y)
        V = _sym(T) if T is not None else np.zeros((n, n))
        Vp = np.maximum(V - np.diag(np.diag(V)), 0.0)
        return float(y.sum() - n * min(0.0, _lmin(np.diag(y) - C - Vp)))
    raise ValueError(kind)


def repaired_primal(kind, A, X):
    """A feasible X built from the primal iterate, and its objective."""
    n = A.shape[0]
    C = objective_matrix(kind, A)
    X = _sym(X)
    if kind in ("maxcut", "cc"):
        Xr = _unit_diag(_psd_part(X))
        if kind == "cc":
            off = Xr - np.eye(n)
            neg = off < 0
            if np.any(neg):
                t = float(np.max(-off[neg] / (1.0 - off[neg])))
                Xr = (1.0 - t) * Xr + t * np.ones((n, n))
    elif kind == "theta":
        E = A > 0.5
        Xr = np.where(E, 0.0, X)
        Xr = Xr + max(0.0, -_lmin(Xr)) * np.eye(n)
        tr = np.trace(Xr)
        Xr = Xr / tr if tr > 0 else np.eye(n) / n
    else:
        raise ValueError(kind)
    return Xr, float(np.sum(C * Xr))


def residuals(kind, A, X, Y, Z, T=None):
    """Primal / dual residual norms of the iterate in the SDP's own variables."""
    n = A.shape[0]
    C = objective_matrix(kind, A)
    X, Y, Z = _sym(X), _sym(Y), _sym(Z)
    if kind in ("maxcut", "cc"):
        rp = np.linalg.norm(np.diag(X) - 1.0)
        Zr = np.diag(np.diag(Y)) - C
        if kind == "cc" and T is not None:
            V = _sym(T)
            Zr = Zr - (V - np.diag(np.diag(V)))
        rd = np.linalg.norm(Z - Zr)
    else:
        E = A > 0.5
        rp = np.sqrt(np.sum(X[E] ** 2) + (np.trace(X) - 1.0) ** 2)
        Zr = Y[0, 0] * np.eye(n) + np.where(E, Y, 0.0) - C
        rd = np.linalg.norm(Z - Zr)
    return float(rp), float(rd)


def certificate(kind, A, X, Y, Z, T=None):
    """Certificate of an iterate (dense matrices in the SDP's variables).

    Returns pobj = C . X, dobj = b^T y, the primal / dual residual norms, the
    smallest eigenvalues of X and Z, the bounds lb <= p* <= ub and the relative
    width (ub - lb) / (1 + |ub|)."""
    C = objective_matrix(kind, A)
    Ys = _sym(Y)
    dobj = float(Ys[0, 0]) if kind == "theta" else float(np.trace(Ys))
    ub = upper_bound(kind, A, Y, T)
    _, lb = repaired_primal(kind, A, X)
    rp, rd = residuals(kind, A, X, Y, Z, T)
    return dict(pobj=float(np.sum(C * _sym(X))), dobj=dobj, res_p=rp, res_d=rd, lmin_x=_lmin(X), lmin_z=_lmin(Z),
                ub=ub, lb=lb, width=(ub - lb) / (1.0 + abs(ub)))


def certificate_tt(kind, A, Xc, Yc, Zc, Tc=None):
    """certificate() of TT iterates given as vec_TT cores (host arrays)."""
    M = dense_matrix
    return certificate(kind, A, M(Xc), M(Yc), M(Zc), M(Tc) if Tc is not None else None)
