"""Plain tensor-train library (oracle; test infrastructure only).

Follows the paper, Sec. 2.3 (Def. "Tensor-Train", "TT Vector", "Interface
Matrix", "Frame Matrix", "TT Matrix", the big-endian vectorisation remark) and
Sec. 3.1/3.3 (Def. "TT Vectorisation", "TT Diagonalisation", the Hadamard
remark and Def. "Kronecker product of TT matrices").  TT rounding is the
QR-then-truncated-SVD method the paper cites (Oseledets 2011).

Representations (all float64 numpy arrays, C order):
  TT vector  : list of cores [r_k, m_k, r_{k+1}]
  TT matrix  : list of cores [R_k, m_out, m_in, R_{k+1}]
Index order is big-endian: core 0 holds the most significant digit, and a
local core [a, i, b] flattens in C order, so vec(T) = T_{!=k} vec(T_k).
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# dense reconstruction
# ----------------------------------------------------------------------------

def full(cores):
    """Dense vector of a TT vector (Def. Tensor-Train, big-endian)."""
    v = np.ones((1, 1))
    for G in cores:
        r, m, s = G.shape
        v = (v @ G.reshape(r, m * s)).reshape(-1, s)
    return v[:, 0]


def full_mat(cores):
    """Dense matrix of a TT matrix (Def. TT Matrix)."""
    M = np.ones((1, 1, 1))
    for G in cores:
        R, mo, mi, S = G.shape
        M = np.einsum("abr,rijs->aibjs", M, G).reshape(M.shape[0] * mo, M.shape[1] * mi, S)
    return M[:, :, 0]


def ranks(cores):
    return [cores[0].shape[0]] + [G.shape[-1] for G in cores]


# ----------------------------------------------------------------------------
# vec_TT, diag_TT, Kronecker, Hadamard (Sec. 3.1 and 3.3)
# ----------------------------------------------------------------------------

def vec_tt(mat_cores):
    """vec_TT of a TT matrix with n x n modes: V_k(s, :, s') = vec(M_k(s, :, :, s'))
    (row-major vec within the mode, the worked example of Def. TT Vectorisation)."""
    return [G.reshape(G.shape[0], G.shape[1] * G.shape[2], G.shape[3]).copy() for G in mat_cores]


def unvec_tt(vec_cores, n=2):
    """Inverse of vec_tt: the TT matrix whose vec_TT is the given TT vector."""
    return [G.reshape(G.shape[0], n, n, G.shape[2]).copy() for G in vec_cores]


def diag_tt(vec_cores):
    """diag_TT: M_k(s, :, :, s') = diag(V_k(s, :, s'))."""
    out = []
    for G in vec_cores:
        r, m, s = G.shape
        D = np.zeros((r, m, m, s))
        for i in range(m):
            D[:, i, i, :] = G[:, i, :]
        out.append(D)
    return out


def kron(A, B):
    """Per-core Kronecker product of two TT matrices (standard Kronecker product
    of 4-way cores): C_k[(a,b), (i,i'), (j,j'), (a',b')] = A_k[a,i,j,a'] B_k[b,i',j',b']."""
    out = []
    for Ga, Gb in zip(A, B):
        ra, mo, mi, sa = Ga.shape
        rb, no, ni, sb = Gb.shape
        C = np.einsum("aijc,bkld->abikjlcd", Ga, Gb).reshape(ra * rb, mo * no, mi * ni, sa * sb)
        out.append(C)
    return out


def transpose_op(A):
    """TT matrix of the transpose: swap output and input mode indices."""
    return [np.ascontiguousarray(G.transpose(0, 2, 1, 3)) for G in A]


def outer(u, v):
    """TT matrix of u v^T from TT vectors u, v."""
    return [np.einsum("aib,cjd->acijbd", Gu, Gv).reshape(Gu.shape[0] * Gv.shape[0], Gu.shape[1],
                                                         Gv.shape[1], Gu.shape[2] * Gv.shape[2])
            for Gu, Gv in zip(u, v)]


def rank1_vec(vectors):
    return [np.asarray(v, dtype=np.float64).reshape(1, -1, 1).copy() for v in vectors]


def rank1_mat(mats):
    return [np.asarray(m, dtype=np.float64).reshape(1, m.shape[0], m.shape[1], 1).copy() for m in mats]


# ----------------------------------------------------------------------------
# linear combinations and products
# ----------------------------------------------------------------------------

def add(cores_list, coeffs):
    """TT of sum_t c_t T_t by block concatenation (vector or matrix cores)."""
    d = len(cores_list[0])
    if d == 1:
        return [sum(c * T[0] for T, c in zip(cores_list, coeffs))]
    out = []
    for k in range(d):
        blocks = [T[k] for T in cores_list]
        mid = blocks[0].shape[1:-1]
        rl = [b.shape[0] for b in blocks]
        rr = [b.shape[-1] for b in blocks]
        if k == 0:
            G = np.concatenate(blocks, axis=-1)
        elif k == d - 1:
            G = np.concatenate([c * b for b, c in zip(blocks, coeffs)], axis=0)
        else:
            G = np.zeros((sum(rl),) + mid + (sum(rr),))
            o1 = o2 = 0
            for b in blocks:
                G[(slice(o1, o1 + b.shape[0]),) + (slice(None),) * len(mid) + (slice(o2, o2 + b.shape[-1]),)] = b
                o1 += b.shape[0]
                o2 += b.shape[-1]
        out.append(G)
    return out


def scale(cores, c):
    out = [G.copy() for G in cores]
    out[-1] = out[-1] * c
    return out


def matvec(A, x):
    """TT matrix times TT vector: cores [R r, m_out, R' r']."""
    out = []
    for Ga, Gx in zip(A, x):
        R, mo, mi, S = Ga.shape
        r, m, s = Gx.shape
        assert m == mi
        out.append(np.einsum("aijc,bjd->abicd", Ga, Gx).reshape(R * r, mo, S * s))
    return out


def matmat(A, B):
    """TT matrix product A B."""
    out = []
    for Ga, Gb in zip(A, B):
        R, mo, mi, S = Ga.shape
        r, no, ni, s = Gb.shape
        assert mi == no
        out.append(np.einsum("aijc,bjkd->abikcd", Ga, Gb).reshape(R * r, mo, ni, S * s))
    return out


def dot(x, y):
    """<x, y> of two TT vectors by left-to-right contraction."""
    E = np.ones((1, 1))
    for Gx, Gy in zip(x, y):
        E = np.einsum("ab,aic,bid->cd", E, Gx, Gy)
    return float(E[0, 0])


def norm(x):
    return float(np.sqrt(max(dot(x, x), 0.0)))


def sandwich(u, A, v):
    """u^T A v for TT vectors u, v and TT matrix A."""
    E = np.ones((1, 1, 1))
    for Gu, Ga, Gv in zip(u, A, v):
        E = np.einsum("abc,aid,bije,cjf->def", E, Gu, Ga, Gv)
    return float(E[0, 0, 0])


# ----------------------------------------------------------------------------
# orthogonalisation, TT-SVD and rounding (Oseledets 2011)
# ----------------------------------------------------------------------------

def _as3(G):
    return G.reshape(G.shape[0], -1, G.shape[-1])


def orth_left(cores, upto=None):
    """Left-orthogonalise cores 0..upto-1 by QR, pushing R into the next core."""
    cores = [G.copy() for G in cores]
    d = len(cores)
    upto = d - 1 if upto is None else upto
    for k in range(upto):
        G = cores[k]
        shp = G.shape
        r, s = shp[0], shp[-1]
        Q, R = np.linalg.qr(G.reshape(-1, s))
        cores[k] = Q.reshape(shp[:-1] + (Q.shape[1],))
        nxt = cores[k + 1]
        cores[k + 1] = np.tensordot(R, nxt, axes=(1, 0))
    return cores


def orth_right(cores, downto=0):
    """Right-orthogonalise cores d-1..downto+1 by QR of the transposed unfolding."""
    cores = [G.copy() for G in cores]
    d = len(cores)
    for k in range(d - 1, downto, -1):
        G = cores[k]
        shp = G.shape
        r = shp[0]
        Q, R = np.linalg.qr(G.reshape(r, -1).T)
        cores[k] = Q.T.reshape((Q.shape[1],) + shp[1:])
        prv = cores[k - 1]
        cores[k - 1] = np.tensordot(prv, R.T, axes=(prv.ndim - 1, 0))
    return cores


def _trunc_rank(s, eps_abs, max_rank):
    """Smallest rank whose discarded tail has Frobenius norm <= eps_abs."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]   # tail[j] = ||s[j:]||
    r = len(s)
    for j in range(1, len(s) + 1):
        t = tail[j] if j < len(s) else 0.0
        if t <= eps_abs:
            r = j
            break
    r = max(1, min(r, max_rank))
    disc = float(np.sqrt(np.sum(s[r:] ** 2)))
    return r, disc


def round_tt(cores, tol, mode="abs", max_rank=1 << 30):
    """TT rounding: right-to-left QR, then left-to-right truncated SVD with the
    per-bond budget tol_abs / sqrt(d - 1).  mode 'rel' scales tol by ||T||_F.
    Returns (rounded cores, zeta) where zeta = ||T - T~||_F is accumulated
    exactly from the discarded singular values (the truncation errors of the
    sweep are mutually orthogonal)."""
    d = len(cores)
    if d == 1:
        return [G.copy() for G in cores], 0.0
    cores = orth_right(cores, 0)
    nrm = float(np.linalg.norm(cores[0]))
    eps = tol * nrm if mode == "rel" else tol
    eps_k = eps / np.sqrt(d - 1)
    zeta2 = 0.0
    out = []
    for k in range(d - 1):
        G = cores[k]
        shp = G.shape
        U, s, Vt = np.linalg.svd(G.reshape(-1, shp[-1]), full_matrices=False)
        r, disc = _trunc_rank(s, eps_k, max_rank)
        zeta2 += disc ** 2
        out.append(U[:, :r].reshape(shp[:-1] + (r,)))
        SV = s[:r, None] * Vt[:r]
        cores[k + 1] = np.tensordot(SV, cores[k + 1], axes=(1, 0))
    out.append(cores[-1])
    return out, float(np.sqrt(zeta2))


def tt_svd(vec, modes, tol=1e-14, max_rank=1 << 30):
    """TT-SVD of a dense vector with the given mode sizes (relative tolerance)."""
    d = len(modes)
    eps_k = tol * np.linalg.norm(vec) / np.sqrt(max(d - 1, 1))
    cores = []
    r = 1
    C = np.asarray(vec, dtype=np.float64).reshape(1, -1)
    for k in range(d - 1):
        C = C.reshape(r * modes[k], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk, _ = _trunc_rank(s, eps_k, max_rank)
        cores.append(U[:, :rk].reshape(r, modes[k], rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, modes[-1], 1))
    return cores


# ----------------------------------------------------------------------------
# interfaces, frames and environments (Defs. Interface/Frame Matrix)
# ----------------------------------------------------------------------------

def interface_left(cores, k):
    """T^{<k} as a dense matrix [prod_{j<k} m_j, r_k]."""
    M = np.ones((1, 1))
    for G in cores[:k]:
        r, m, s = G.shape
        M = (M @ G.reshape(r, m * s)).reshape(-1, s)
    return M


def interface_right(cores, k):
    """T^{>k} as a dense matrix [prod_{j>k} m_j, r_{k+1}]."""
    M = np.ones((1, 1))        # [r_{d}, 1] style accumulator: rows = right index
    for G in reversed(cores[k + 1:]):
        r, m, s = G.shape
        M = (G.reshape(r * m, s) @ M.reshape(s, -1)).reshape(r, -1)
    return M.T


def frame(cores, k):
    """Frame matrix T_{!=k} = T^{<k} kron I_{m_k} kron T^{>k}."""
    m = cores[k].shape[1]
    return np.kron(np.kron(interface_left(cores, k), np.eye(m)), interface_right(cores, k))


def env_left_step(phi, V, O, U):
    """Phi'[a2, beta, c2] = sum V[a,i,a2] Phi[a,alpha,c] O[alpha,i,j,beta] U[c,j,c2].
    O None means the identity (then phi has a unit middle index)."""
    if O is None:
        t = np.tensordot(phi[:, 0, :], U, axes=([1], [0]))          # [a, i, c2]
        return np.tensordot(V, t, axes=([0, 1], [0, 1]))[:, None, :]  # [a2, 1, c2]
    t1 = np.tensordot(phi, U, axes=([2], [0]))                       # [a, alpha, j, c2]
    t2 = np.tensordot(t1, O, axes=([1, 2], [0, 2]))                  # [a, c2, i, beta]
    out = np.tensordot(V, t2, axes=([0, 1], [0, 2]))                 # [a2, c2, beta]
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def env_right_step(phi, V, O, U):
    """Phi'[a, alpha, c] = sum V[a,i,a2] O[alpha,i,j,beta] U[c,j,c2] Phi[a2,beta,c2]."""
    if O is None:
        t = np.tensordot(U, phi[:, 0, :], axes=([2], [1]))            # [c, i, a2]
        return np.tensordot(V, t, axes=([1, 2], [1, 2]))[:, None, :]  # [a, 1, c]
    t1 = np.tensordot(U, phi, axes=([2], [2]))                       # [c, j, a2, beta]
    t2 = np.tensordot(t1, O, axes=([1, 3], [2, 3]))                  # [c, a2, alpha, i]
    out = np.tensordot(V, t2, axes=([1, 2], [3, 1]))                 # [a, c, alpha]
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def envs(V, O, U):
    """All left and right environments of the triple (test V, operator O, trial U).
    left[k] contracts cores < k, right[k] contracts cores > k."""
    d = len(V)
    one = np.ones((1, 1, 1))
    left = [one]
    for k in range(d - 1):
        left.append(env_left_step(left[-1], V[k], None if O is None else O[k], U[k]))
    right = [None] * d
    right[d - 1] = one
    for k in range(d - 1, 0, -1):
        right[k - 1] = env_right_step(right[k], V[k], None if O is None else O[k], U[k])
    return left, right


def local_apply(phiL, O, x, phiR):
    """Projected local action y[a,i,b] = sum phiL[a,al,a'] O[al,i,j,be] x[a',j,b'] phiR[b,be,b']."""
    if O is None:
        t = np.tensordot(phiL[:, 0, :], x, axes=([1], [0]))          # [a, j, b']
        return np.tensordot(t, phiR[:, 0, :], axes=([2], [1]))       # [a, j, b]
    t1 = np.tensordot(phiL, x, axes=([2], [0]))                      # [a, al, j, b']
    t2 = np.tensordot(t1, O, axes=([1, 2], [0, 2]))                  # [a, b', i, be]
    return np.tensordot(t2, phiR, axes=([3, 1], [1, 2]))             # [a, i, b]


def local_dense(phiL, O, phiR):
    """Dense projected operator [(a,i,b), (a',j,b')] from environments."""
    t = np.tensordot(phiL, O, axes=([1], [0]))                       # [a, a', i, j, be]
    M = np.tensordot(t, phiR, axes=([4], [1]))                       # [a, a', i, j, b, b']
    M = M.transpose(0, 2, 4, 1, 3, 5)
    a, i, b = M.shape[:3]
    return np.ascontiguousarray(M).reshape(a * i * b, -1)
