"""Dense Newton systems of the TT interior-point method (oracle; test only).

Builds, densely and in the padded vec_TT index space of Sec. 3.2/3.3, the
block Newton system of eq. (tt-kkt-newton-system):

    [ 0          -Aeq^T   -s Aineq^T       I   ] [dX]     [R_d]
    [ -Aeq        K_Y      0               0   ] [dY] = - [R_p]
    [ -s T Aineq  0        D_ineq(X) + K_T 0   ] [dT]     [R_t]
    [ L_Z         0        0               L_X ] [dZ]     [R_c]

with s = +1 for A_ineq X <= B_ineq and s = -1 for the >= convention of the
correlation-clustering formulation (Sec. 4.3), and the residuals

    R_d = Z + C - Aeq^T Y - s Aineq^T T,   R_p = B_eq - Aeq X,
    R_t = T o s_ineq(X) - mu 1_T,          s_ineq(X) = s (B_ineq - Aineq X),
    R_c = L_Z X - 2 mu I  (AHO),  (Z x I) X - mu I  (XZ warm-up).

AHO: L_Z = I x Z + Z x I, L_X = I x X + X x I; XZ: L_Z = Z x I, L_X = I x X
(per-core Kronecker products, Def. "Kronecker product of TT matrices", so that
(A x B) vec_TT(M) = vec_TT(A M B^T)).  The dense solve is by LU.
"""
from __future__ import annotations

import numpy as np

from . import tt


def identity_mat_tt(d):
    return tt.rank1_mat([np.eye(2)] * d)


def L_ops(X, Z, direction):
    """TT operators (L_Z, L_X) for the AHO or XZ direction from vec_TT X, Z."""
    d = len(X)
    I = identity_mat_tt(d)
    Xm, Zm = tt.unvec_tt(X), tt.unvec_tt(Z)
    if direction == "aho":
        LZ = tt.add([tt.kron(I, Zm), tt.kron(Zm, I)], [1.0, 1.0])
        LX = tt.add([tt.kron(I, Xm), tt.kron(Xm, I)], [1.0, 1.0])
    elif direction == "xz":
        LZ = tt.kron(Zm, I)
        LX = tt.kron(I, Xm)
    else:
        raise ValueError(direction)
    return LZ, LX


def one_T(prob):
    """vec_TT of 1_T: ones on active inequality positions (I - K_T applied to J)."""
    d = prob["d"]
    J = tt.rank1_vec([np.ones(4)] * d)
    return tt.add([J, tt.matvec(prob["KT"], J)], [1.0, -1.0])


def residuals_dense(prob, X, Y, Z, T, mu, direction, sigma_mu=None):
    """Dense residual vectors (R_d, R_p, R_t, R_c) in vec_TT order."""
    f = tt.full
    Aeq, AeqT = tt.full_mat(prob["Aeq"]), tt.full_mat(prob["AeqT"])
    x, y, z = f(X), f(Y), f(Z)
    Rd = z + f(prob["C"]) - AeqT @ y
    Rp = f(prob["Beq"]) - Aeq @ x
    Rt = None
    if "Aineq" in prob:
        s = prob["sense"]
        AiT, Ai = tt.full_mat(prob["AineqT"]), tt.full_mat(prob["Aineq"])
        t = f(T)
        Rd = Rd - s * (AiT @ t)
        slack = s * (f(prob["Bineq"]) - Ai @ x)
    target = mu if sigma_mu is None else sigma_mu
    if "Aineq" in prob:
        # both complementarity residuals aim at the same target (0 for the
        # affine predictor, sigma mu for the corrector)
        Rt = t * slack - target * f(one_T(prob))
    LZ, LX = L_ops(X, Z, direction)
    Ivec = f(tt.rank1_vec([np.array([1.0, 0, 0, 1])] * prob["d"]))
    coef = 2.0 if direction == "aho" else 1.0
    Rc = tt.full_mat(LZ) @ x - coef * target * Ivec
    return Rd, Rp, Rt, Rc


def newton_dense(prob, X, Y, Z, T, mu, direction, Rc_override=None, sigma_mu=None, Rt_override=None):
    """Solve the dense block Newton system; returns dense (dX, dY, dT, dZ)."""
    f = tt.full
    N2 = 4 ** prob["d"]
    Aeq, AeqT = tt.full_mat(prob["Aeq"]), tt.full_mat(prob["AeqT"])
    KY = tt.full_mat(prob["KY"])
    LZ, LX = L_ops(X, Z, direction)
    LZd, LXd = tt.full_mat(LZ), tt.full_mat(LX)
    Rd, Rp, Rt, Rc = residuals_dense(prob, X, Y, Z, T, mu, direction, sigma_mu)
    if Rc_override is not None:
        Rc = Rc_override
    if Rt_override is not None:
        Rt = Rt_override
    I = np.eye(N2)
    O = np.zeros((N2, N2))
    if "Aineq" not in prob:
        K = np.block([[O, -AeqT, I], [-Aeq, KY, O], [LZd, O, LXd]])
        rhs = -np.concatenate([Rd, Rp, Rc])
        sol = np.linalg.solve(K, rhs)
        dX, dY, dZ = np.split(sol, 3)
        return dX, dY, None, dZ
    s = prob["sense"]
    Ai, AiT, KT = tt.full_mat(prob["Aineq"]), tt.full_mat(prob["AineqT"]), tt.full_mat(prob["KT"])
    t = f(T)
    slack = s * (f(prob["Bineq"]) - Ai @ f(X))
    TA = np.diag(t) @ Ai
    D = np.diag(slack)
    K = np.block([[O, -AeqT, -s * AiT, I],
                  [-Aeq, KY, O, O],
                  [-s * TA, O, D + KT, O],
                  [LZd, O, O, LXd]])
    rhs = -np.concatenate([Rd, Rp, Rt, Rc])
    sol = np.linalg.solve(K, rhs)
    dX, dY, dT, dZ = np.split(sol, 4)
    return dX, dY, dT, dZ
