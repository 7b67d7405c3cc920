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

Also here, for a frame matrix W (N x p, orthonormal columns):
  * reduced_system: the projected system of eq. (reduced_kkt_system), dZ
    eliminated before the solve, with the chained products
    (W^T L_X W)(W^T Aeq^T W) kept as products of projections;
  * block_elimination: the solve of that system by the Cholesky factor of
    W^T L_Z W, the LU of Phi and of the Schur complement S, and the
    triangular solves in the order dY -> dT -> dX of Sec. 3.3;
  * dz_local: the elimination formula for dZ_k of Sec. 3.3.
With W = I the reduced system is the full system with dZ substituted.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

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


def system_blocks(prob, X, Y, Z, T, mu, direction, Rc_override=None, sigma_mu=None, Rt_override=None):
    """Dense operator blocks and residuals of eq. (tt-kkt-newton-system).

    Returns a dict with Aeq, AeqT, KY, LZ, LX (N x N), the residuals Rd, Rp,
    Rc (and Rt), and for inequalities Ai, AiT, TA (= diag_TT(vec T) Aineq),
    DK (= D_ineq(X) + K_T) and the sense s."""
    f = tt.full
    B = dict(ineq="Aineq" in prob)
    B["Aeq"], B["AeqT"] = tt.full_mat(prob["Aeq"]), tt.full_mat(prob["AeqT"])
    B["KY"] = tt.full_mat(prob["KY"])
    LZ, LX = L_ops(X, Z, direction)
    B["LZ"], B["LX"] = tt.full_mat(LZ), tt.full_mat(LX)
    Rd, Rp, Rt, Rc = residuals_dense(prob, X, Y, Z, T, mu, direction, sigma_mu)
    B["Rd"], B["Rp"] = Rd, Rp
    B["Rc"] = Rc if Rc_override is None else Rc_override
    if B["ineq"]:
        s = prob["sense"]
        B["s"] = s
        B["Ai"], B["AiT"] = tt.full_mat(prob["Aineq"]), tt.full_mat(prob["AineqT"])
        B["TA"] = np.diag(f(T)) @ B["Ai"]
        slack = s * (f(prob["Bineq"]) - B["Ai"] @ f(X))
        B["DK"] = np.diag(slack) + tt.full_mat(prob["KT"])
        B["Rt"] = Rt if Rt_override is None else Rt_override
    return B


def assemble(B):
    """The unreduced block matrix K and right-hand side -R (unknowns dX, dY, [dT,] dZ)."""
    N = B["Aeq"].shape[0]
    I = np.eye(N)
    O = np.zeros((N, N))
    if not B["ineq"]:
        K = np.block([[O, -B["AeqT"], I], [-B["Aeq"], B["KY"], O], [B["LZ"], O, B["LX"]]])
        R = np.concatenate([B["Rd"], B["Rp"], B["Rc"]])
        return K, -R
    s = B["s"]
    K = np.block([[O, -B["AeqT"], -s * B["AiT"], I],
                  [-B["Aeq"], B["KY"], O, O],
                  [-s * B["TA"], O, B["DK"], O],
                  [B["LZ"], O, O, B["LX"]]])
    R = np.concatenate([B["Rd"], B["Rp"], B["Rt"], B["Rc"]])
    return K, -R


def newton_dense(prob, X, Y, Z, T, mu, direction, Rc_override=None, sigma_mu=None, Rt_override=None):
    """Solve the dense block Newton system; returns dense (dX, dY, dT, dZ)."""
    B = system_blocks(prob, X, Y, Z, T, mu, direction, Rc_override, sigma_mu, Rt_override)
    K, rhs = assemble(B)
    sol = np.linalg.solve(K, rhs)
    if not B["ineq"]:
        dX, dY, dZ = np.split(sol, 3)
        return dX, dY, None, dZ
    dX, dY, dT, dZ = np.split(sol, 4)
    return dX, dY, dT, dZ


def _proj(W, A):
    return W.T @ A @ W


def reduced_system(B, W):
    """Eq. (reduced_kkt_system) for the frame W: matrix and right-hand side in
    the unknowns (dX_k, dY_k[, dT_k]); dZ_k has been eliminated."""
    Ah, ATh, KYh = _proj(W, B["Aeq"]), _proj(W, B["AeqT"]), _proj(W, B["KY"])
    LZh, LXh = _proj(W, B["LZ"]), _proj(W, B["LX"])
    Rdh, Rph, Rch = W.T @ B["Rd"], W.T @ B["Rp"], W.T @ B["Rc"]
    p = W.shape[1]
    O = np.zeros((p, p))
    if not B["ineq"]:
        K = np.block([[-Ah, KYh], [LZh, LXh @ ATh]])
        rhs = -np.concatenate([Rph, Rch - LXh @ Rdh])
        return K, rhs
    s = B["s"]
    TAh, DKh, AiTh = _proj(W, B["TA"]), _proj(W, B["DK"]), _proj(W, B["AiT"])
    Rth = W.T @ B["Rt"]
    # the inequality blocks carry the sense s of the >= convention exactly as
    # in the unreduced system (-s T Aineq in row t, -s Aineq^T in row d)
    K = np.block([[-Ah, KYh, O], [-s * TAh, O, DKh], [LZh, LXh @ ATh, s * (LXh @ AiTh)]])
    rhs = -np.concatenate([Rph, Rth, Rch - LXh @ Rdh])
    return K, rhs


def dz_local(B, W, dY, dT=None):
    """dZ_k = W^T Aeq^T W dY_k (+ s W^T Aineq^T W dT_k) - W^T R_d (Sec. 3.3)."""
    dz = _proj(W, B["AeqT"]) @ dY - W.T @ B["Rd"]
    if B["ineq"]:
        dz = dz + B["s"] * (_proj(W, B["AiT"]) @ dT)
    return dz


def block_elimination(B, W):
    """Sec. 3.3 block elimination on the frame W: Cholesky of L_Z^, LU of Phi
    and of the Schur complement S, then dY, dT, dX by triangular solves.
    Returns (dX_k, dY_k, dT_k or None, dZ_k)."""
    Ah, ATh, KYh = _proj(W, B["Aeq"]), _proj(W, B["AeqT"]), _proj(W, B["KY"])
    LZh, LXh = _proj(W, B["LZ"]), _proj(W, B["LX"])
    Rdh, Rph, Rch = W.T @ B["Rd"], W.T @ B["Rp"], W.T @ B["Rc"]
    cz = sla.cho_factor(0.5 * (LZh + LZh.T), lower=True)
    LZinv = lambda M: sla.cho_solve(cz, M)
    # g = L_Z^{-1} (L_X^ R_d^ - R_c^)
    g = LZinv(LXh @ Rdh - Rch)
    if not B["ineq"]:
        S = Ah @ LZinv(LXh @ ATh) + KYh
        dY = sla.lu_solve(sla.lu_factor(S), Ah @ g - Rph)
        dT = None
        dZ = dz_local(B, W, dY)
    else:
        s = B["s"]
        TAh, DKh, AiTh = _proj(W, B["TA"]), _proj(W, B["DK"]), _proj(W, B["AiT"])
        Rth = W.T @ B["Rt"]
        # With the sense s the t row reads -s TA^ dX + DK^ dT = -R_t^ and the
        # chained block is s L_X^ Aineq^T^; eliminating dX = -L_Z^{-1}(L_X^ Aeq^T^ dY
        # + s L_X^ Aineq^T^ dT) + g gives
        #   Phi dT = s TA^ (g - L_Z^{-1} L_X^ Aeq^T^ dY) - R_t^,
        #   Phi    = DK^ + s^2 TA^ L_Z^{-1} L_X^ Aineq^T^,
        # and for dY the Schur complement of Phi in the (y, t) system.
        G_y = LZinv(LXh @ ATh)
        G_t = LZinv(LXh @ AiTh)
        Phi = DKh + (s * s) * TAh @ G_t
        luP = sla.lu_factor(Phi)
        Pinv = lambda M: sla.lu_solve(luP, M)
        # y row: -A^ dX + KY^ dY = -R_p^ with dX as above:
        #   (A^ G_y + KY^) dY + s A^ G_t dT = A^ g - R_p^
        # t row: Phi dT + s TA^ G_y dY = s TA^ g - R_t^
        S = Ah @ G_y + KYh - (s * s) * Ah @ G_t @ Pinv(TAh @ G_y)
        rhs_y = Ah @ g - Rph - s * Ah @ G_t @ Pinv(s * TAh @ g - Rth)
        dY = sla.lu_solve(sla.lu_factor(S), rhs_y)
        dT = Pinv(s * TAh @ (g - G_y @ dY) - Rth)
        dZ = dz_local(B, W, dY, dT)
    dX = -LZinv(Rch + LXh @ dZ)
    return dX, dY, dT, dZ
