"""The paper's SDP encodings in TT form and as dense data (oracle; test only).

TT encodings follow Sec. 4 (Maximum Cut, Maximum Stable Set, Correlation
Clustering) with the elementary TT matrices I, J and E_(alpha;beta) of the same
section, vec_TT / diag_TT of Sec. 3.1/3.3, and the padded multipliers and masks
K_Y, K_T of Sec. 3.2/3.3.  Dense data follow the SDP relaxations of Sec. 2.2
(Examples "Maximum Cut", "Maximum Stable Set", "Correlation Clustering").

A TT problem is a dict with
  kind, d, n (= 2^d), C (vec_TT of the objective, TT vector with mode 4),
  Aeq, AeqT, KY (TT matrices with 4 x 4 modes), Beq (TT vector),
  and for inequalities Aineq, AineqT, KT, Bineq, sense (+1 for <=, -1 for >=),
  m (number of equality constraints) and q (number of stored, mirrored
  inequality multipliers).
"""
from __future__ import annotations

import numpy as np

from . import tt

_I4 = np.array([1.0, 0.0, 0.0, 1.0])   # vec of the 2x2 identity (row-major)
_J4 = np.array([1.0, 1.0, 1.0, 1.0])   # vec of the 2x2 all-ones matrix
_E4 = np.array([1.0, 0.0, 0.0, 0.0])   # vec of E_11 (2x2)


def _const_vec(v, d):
    return tt.rank1_vec([v] * d)


def maxcut(A_cores):
    """MaxCut in TT (Sec. 4.1): C = (diag_TT(A_G 1) - A_G) / 4,
    A_eq = diag_TT(vec_TT I), B_eq = vec_TT I, K_Y = diag_TT(vec_TT(J - I))."""
    d = len(A_cores)
    deg = [G.sum(axis=2) for G in A_cores]           # A_G 1 as a TT vector (mode 2)
    C = tt.add([tt.diag_tt(deg), A_cores], [0.25, -0.25])
    Ivec = _const_vec(_I4, d)
    Jvec = _const_vec(_J4, d)
    Aeq = tt.diag_tt(Ivec)
    return dict(kind="maxcut", d=d, n=2 ** d, C=tt.vec_tt(C), Aeq=Aeq, AeqT=Aeq, Beq=Ivec,
                KY=tt.diag_tt(tt.add([Jvec, Ivec], [1.0, -1.0])), m=2 ** d, q=0,
                lam0=1.0)


def theta(A_cores):
    """Lovasz theta in TT (Sec. 4.2): C = J,
    A_eq = diag_TT(vec_TT A_G) + vec_TT(E_11) vec_TT(I)^T, B_eq = vec_TT(E_11),
    K_Y = diag_TT(vec_TT(J - A_G) - B_eq)  (graph weights must be 0/1)."""
    d = len(A_cores)
    Ivec = _const_vec(_I4, d)
    Jvec = _const_vec(_J4, d)
    Evec = _const_vec(_E4, d)
    Avec = tt.vec_tt(A_cores)
    part1 = tt.diag_tt(Avec)
    Aeq = tt.add([part1, tt.outer(Evec, Ivec)], [1.0, 1.0])
    AeqT = tt.add([part1, tt.outer(Ivec, Evec)], [1.0, 1.0])
    KY = tt.diag_tt(tt.add([Jvec, Avec, Evec], [1.0, -1.0, -1.0]))
    nedges = int(round(tt.dot(Avec, Jvec)))
    return dict(kind="theta", d=d, n=2 ** d, C=Jvec, Aeq=Aeq, AeqT=AeqT, Beq=Evec, KY=KY,
                m=nedges // 2 + 1, q=0, lam0=2.0)


def cc(W_cores, negdeg_cores):
    """Correlation clustering in TT (Sec. 4.3) with E = all off-diagonal pairs:
    C = C+ + diag_TT(C- 1) - C- = W + diag_TT(C- 1) (W = C+ - C-),
    A_eq = diag_TT(vec_TT I), B_eq = vec_TT I, K_Y = diag_TT(vec_TT(J - I)),
    A_ineq = diag_TT(vec_TT(J - I)) with the >= convention (s = A_ineq vec X),
    K_T = diag_TT(vec_TT I).  negdeg_cores is the TT vector (mode 2) of C- 1."""
    d = len(W_cores)
    C = tt.add([W_cores, tt.diag_tt(negdeg_cores)], [1.0, 1.0])
    Ivec = _const_vec(_I4, d)
    Jvec = _const_vec(_J4, d)
    AGvec = tt.add([Jvec, Ivec], [1.0, -1.0])
    Aeq = tt.diag_tt(Ivec)
    Aineq = tt.diag_tt(AGvec)
    n = 2 ** d
    return dict(kind="cc", d=d, n=n, C=tt.vec_tt(C), Aeq=Aeq, AeqT=Aeq, Beq=Ivec,
                KY=tt.diag_tt(AGvec), Aineq=Aineq, AineqT=Aineq, KT=tt.diag_tt(Ivec),
                Bineq=tt.scale(Ivec, 0.0), sense=-1.0, m=n, q=n * n - n, lam0=2.0)


# ----------------------------------------------------------------------------
# dense data for the dense IPM (Sec. 2.2 examples)
# ----------------------------------------------------------------------------

def maxcut_dense(A):
    """max (1/4) L . X  s.t. diag X = 1, X psd;  L = Diag(A 1) - A."""
    n = A.shape[0]
    L = np.diag(A.sum(axis=1)) - A
    return dict(n=n, C=0.25 * L, eq=[("diag", np.arange(n), np.ones(n))], ineq=[])


def theta_dense(A):
    """max J . X  s.t. tr X = 1, X_uv = 0 on edges, X psd."""
    n = A.shape[0]
    iu, ju = np.nonzero(np.triu(A, 1))
    return dict(n=n, C=np.ones((n, n)),
                eq=[("trace", None, np.ones(1)), ("pair", (iu, ju), np.zeros(len(iu)))], ineq=[])


def cc_dense(W):
    """max (C+ + L-) . X s.t. diag X = 1, X_uv >= 0 for all pairs u < v, X psd."""
    n = W.shape[0]
    Cm = np.maximum(-W, 0.0)
    C = W + np.diag(Cm.sum(axis=1))
    iu, ju = np.triu_indices(n, 1)
    return dict(n=n, C=C, eq=[("diag", np.arange(n), np.ones(n))],
                ineq=[("pair", (iu, ju), np.zeros(len(iu)))])
