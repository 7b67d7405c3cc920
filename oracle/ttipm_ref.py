"""Reference TT interior-point method (oracle; test infrastructure only).

A plain NumPy rendering of the paper's TT-IPM, step by step in the paper's
order and notation:

  * Alg. 1 (primal-dual IPM loop) with mu of Sec. 3.3, the residuals R_d, R_p,
    R_t, R_c of eq. (tt-kkt-newton-system), Mehrotra's predictor-corrector
    (Sec. 3.5) and the XZ warm-up followed by the AHO direction (Sec. 3.3/5.1);
  * the Newton system solved by a block-AMEn sweep over a block TT that holds
    dX, dY, [dT], dZ in one shared frame (Sec. 2.3 Def. "Block Tensor-Train",
    Sec. 3.3): local elimination of dZ, the reduced projected system of eq.
    (reduced_kkt_system) with the chained products L_X^ Aeq^T^, the block index
    moved by SVD, cached left/right environments (never the frame matrix);
  * TT rounding with the spectral shift of Cor. 1 (Sec. 3.4) and the tolerance
    schedule eta <- max(min(eta, C mu), delta) of Sec. 3.5;
  * step lengths from the definition of Thm. 1 on dense matrices (small n only;
    this is the quantity the TT eigen-solver of Sec. 3.4 approximates).

Local systems are solved densely (numpy.linalg.solve) so that every local
solution is exact; this is the slow, obviously correct counterpart of the
library's Krylov solver.  Readings of points the paper leaves open are marked
"reading:" in the comments.

Pins: at full TT rank the solve reaches the closed-form SDP values of K_8 and
C_7 + K_1 (MaxCut) and of C_5 + 3 K_1 (theta), tests/test_oracle_ttipm_ref.py.
Under binding rank caps nothing pins it: its enrichment and its capped
rounding with the Cor. 1 shift follow the same readings as the library, so it
cannot tell a defect of those readings from behaviour of the method.
"""
from __future__ import annotations

import math
import time
import numpy as np

from . import tt
from .kkt import L_ops, one_T, identity_mat_tt

I4 = np.array([1.0, 0.0, 0.0, 1.0])


def _ivec(d):
    return tt.rank1_vec([I4] * d)


# ----------------------------------------------------------------------------
# block TT helpers
# ----------------------------------------------------------------------------

class BlockTT:
    """Shared-frame block TT: cores[k] for k != pos are [r, 4, r']; the block
    core at `pos` is stored component-major as blk[L'][r_pos][4][r_pos+1]."""

    def __init__(self, cores, pos, blk):
        self.cores = cores
        self.pos = pos
        self.blk = blk

    @property
    def d(self):
        return len(self.cores)

    def component(self, l):
        out = [None if G is None else G.copy() for G in self.cores]
        out[self.pos] = self.blk[l].copy()
        return out

    def ranks(self):
        return tt.ranks(self.component(0))


def _kick(U, rho, rng, cap=1 << 30):
    """Enrichment (Sec. 2.3, AMEn): append rho orthonormal columns orthogonal to
    U.  reading: the columns are random (a seeded Gaussian kick) rather than
    residual cores; they make the frame grow so that the block-ALS fixed point
    is the Newton solution and the local residual test detects missing
    directions.  They only fill the capacity left under the rank cap."""
    rows, rk = U.shape
    q = min(rho, rows - rk, cap - rk)
    if q <= 0:
        return U
    G = rng.standard_normal((rows, q))
    for _ in range(2):
        G = G - U @ (U.T @ G)
    Q, _ = np.linalg.qr(G)
    return np.hstack([U, Q])


def _split_left(blk, tol_rel, rank_cap, weights, kick=0, rng=None):
    """SVD move of the block index to the right neighbour (Sec. 2.3): the matrix
    M[(a,i), (l,b)] gives a left-orthonormal U (truncated); coefficients U^T M.
    reading: truncation is taken on the component-normalised matrix so that a
    small component is not lost next to a large one."""
    Lp, r, m, s = blk.shape
    M = blk.transpose(1, 2, 0, 3).reshape(r * m, Lp * s)
    Ms = (blk / weights[:, None, None, None]).transpose(1, 2, 0, 3).reshape(r * m, Lp * s)
    U, sv, _ = np.linalg.svd(Ms, full_matrices=False)
    rk = _rank_for(sv, tol_rel, max(1, rank_cap))
    U = U[:, :rk]
    if kick:
        U = _kick(U, kick, rng, rank_cap)
    rk = U.shape[1]
    coef = U.T @ M                                   # [rk, (l, b)]
    return U.reshape(r, m, rk), coef.reshape(rk, Lp, s)


def _split_right(blk, tol_rel, rank_cap, weights, kick=0, rng=None):
    """Block index moved to the left neighbour: M[(a,l), (i,b)] = V^T rows."""
    Lp, r, m, s = blk.shape
    M = blk.transpose(1, 0, 2, 3).reshape(r * Lp, m * s)
    Ms = (blk / weights[:, None, None, None]).transpose(1, 0, 2, 3).reshape(r * Lp, m * s)
    _, sv, Vt = np.linalg.svd(Ms, full_matrices=False)
    rk = _rank_for(sv, tol_rel, max(1, rank_cap))
    V = Vt[:rk].T                                    # [(i,b), rk]
    if kick:
        V = _kick(V, kick, rng, rank_cap)
    rk = V.shape[1]
    coef = M @ V                                     # [(a,l), rk]
    return V.T.reshape(rk, m, s), coef.reshape(r, Lp, rk)


def _weights(blk):
    """Per-component norms used to normalise the block before its SVD; a
    component at rounding level relative to the largest keeps the largest
    weight (normalising pure rounding noise would inflate the rank)."""
    w = np.array([np.linalg.norm(b) for b in blk])
    wmax = w.max()
    if wmax == 0.0:
        return np.ones_like(w)
    return np.where(w > 1e-8 * wmax, w, wmax)


def _rank_for(sv, tol_rel, cap):
    if sv[0] == 0.0:
        return 1
    tot = np.sqrt(np.sum(sv ** 2))
    tail = np.sqrt(np.cumsum((sv ** 2)[::-1]))[::-1]
    rk = len(sv)
    for j in range(1, len(sv)):
        if tail[j] <= tol_rel * tot:
            rk = j
            break
    return max(1, min(rk, cap))


# ----------------------------------------------------------------------------
# the Newton system in block-AMEn form
# ----------------------------------------------------------------------------

class NewtonSystem:
    """Operators and right-hand-side terms of the reduced projected system.

    Solved components: 0 = dX, 1 = dY, 2 = dT (with inequalities); the last
    stored component is dZ, eliminated locally (Sec. 3.3):
        vec dZ_k = Aeq^T^ dY_k + s Aineq^T^ dT_k - R_d^.
    Residual terms are lists of (coefficient, operator name or None, TT vector)."""

    def __init__(self, prob, ops, rd, rp, rc, rt=None):
        self.prob = prob
        self.ops = ops            # name -> TT matrix (4 x 4 modes)
        self.rd, self.rp, self.rc, self.rt = rd, rp, rc, rt
        self.ineq = "Aineq" in prob
        self.L = 3 if self.ineq else 2
        self.s = prob.get("sense", 1.0)


def _all_terms(sysm):
    terms = []
    for name in ("rd", "rp", "rc", "rt"):
        lst = getattr(sysm, name)
        if lst:
            for (c, op, v) in lst:
                terms.append((name, c, op, v))
    return terms


class Envs:
    """Cached left/right environments for every (operator, trial) pair."""

    def __init__(self, sysm, W):
        self.sysm = sysm
        d = W.d
        self.d = d
        self.sys_ops = list(sysm.ops.keys())
        self.terms = _all_terms(sysm)
        one = np.ones((1, 1, 1))
        self.L = {key: [None] * d for key in self._keys()}
        self.R = {key: [None] * d for key in self._keys()}
        for key in self._keys():
            self.L[key][0] = one
            self.R[key][d - 1] = one

    def _keys(self):
        keys = [("op", n) for n in self.sys_ops]
        keys += [("term", i) for i in range(len(self.terms))]
        return keys

    def _op_trial(self, key, W, k):
        if key[0] == "op":
            return self.sysm.ops[key[1]][k], W.cores[k]
        name, c, op, v = self.terms[key[1]]
        return (None if op is None else self.sysm.ops[op][k]), v[k]

    def update_left(self, W, k):
        for key in self._keys():
            O, U = self._op_trial(key, W, k)
            self.L[key][k + 1] = tt.env_left_step(self.L[key][k], W.cores[k], O, U)

    def update_right(self, W, k):
        for key in self._keys():
            O, U = self._op_trial(key, W, k)
            self.R[key][k - 1] = tt.env_right_step(self.R[key][k], W.cores[k], O, U)


def _local_op(envs, name, k):
    O = envs.sysm.ops[name][k]
    return tt.local_dense(envs.L[("op", name)][k], O, envs.R[("op", name)][k])


def _local_vec(envs, which, k, shape):
    out = np.zeros(shape)
    for i, (name, c, op, v) in enumerate(envs.terms):
        if name != which:
            continue
        O = None if op is None else envs.sysm.ops[op][k]
        out += c * tt.local_apply(envs.L[("term", i)][k], O, v[k], envs.R[("term", i)][k])
    return out


def local_system(envs, k, r, s):
    """Dense reduced projected system (eq. reduced_kkt_system) at core k."""
    sysm = envs.sysm
    p = r * 4 * s
    A = _local_op(envs, "Aeq", k)
    AT = _local_op(envs, "AeqT", k)
    KY = _local_op(envs, "KY", k)
    LZ = _local_op(envs, "LZ", k)
    LX = _local_op(envs, "LX", k)
    shp = (r, 4, s)
    Rd = _local_vec(envs, "rd", k, shp).ravel()
    Rp = _local_vec(envs, "rp", k, shp).ravel()
    Rc = _local_vec(envs, "rc", k, shp).ravel()
    Z0 = np.zeros((p, p))
    if not sysm.ineq:
        K = np.block([[-A, KY], [LZ, LX @ AT]])
        f = np.concatenate([-Rp, -Rc + LX @ Rd])
        parts = dict(AT=AT, Rd=Rd)
        return K, f, parts
    sg = sysm.s
    TA = _local_op(envs, "TA", k)
    DK = _local_op(envs, "DK", k)
    AiT = _local_op(envs, "AineqT", k)
    Rt = _local_vec(envs, "rt", k, shp).ravel()
    K = np.block([[-A, KY, Z0], [-sg * TA, Z0, DK], [LZ, LX @ AT, sg * (LX @ AiT)]])
    f = np.concatenate([-Rp, -Rt, -Rc + LX @ Rd])
    return K, f, dict(AT=AT, AiT=AiT, Rd=Rd)


def local_block_elimination(envs, k, r, s):
    """Direct solve of the reduced system by the paper's block elimination
    (Sec. 3.3): Cholesky of L_Z^, LU of the Schur complement
    S = Aeq^ L_Z^{-1} L_X^ Aeq^T^ + K_Y^ (and of Phi with inequalities),
    then dY_k, [dT_k], dZ_k and dX_k = -L_Z^{-1}(R_c^ + L_X^ dZ_k) in that order."""
    import scipy.linalg as sla
    sysm = envs.sysm
    A = _local_op(envs, "Aeq", k)
    AT = _local_op(envs, "AeqT", k)
    KY = _local_op(envs, "KY", k)
    LZ = _local_op(envs, "LZ", k)
    LX = _local_op(envs, "LX", k)
    shp = (r, 4, s)
    Rd = _local_vec(envs, "rd", k, shp).ravel()
    Rp = _local_vec(envs, "rp", k, shp).ravel()
    Rc = _local_vec(envs, "rc", k, shp).ravel()
    LZs = 0.5 * (LZ + LZ.T)
    cf = sla.cho_factor(LZs)
    if sysm.ineq:
        raise NotImplementedError("block elimination with inequalities")
    G = sla.cho_solve(cf, LX @ AT)                      # L_Z^{-1} L_X^ Aeq^T^
    S = A @ G + KY
    rhs_y = A @ sla.cho_solve(cf, LX @ Rd - Rc) - Rp
    y = np.linalg.solve(S, rhs_y)
    dz = AT @ y - Rd
    x = -sla.cho_solve(cf, Rc + LX @ dz)
    return np.concatenate([x, y]), dz


def _dz_local(sysm, parts, sol, p):
    y = sol[p:2 * p]
    dz = parts["AT"] @ y - parts["Rd"]
    if sysm.ineq:
        dz = dz + sysm.s * (parts["AiT"] @ sol[2 * p:3 * p])
    return dz


def amen_solve(sysm, W, tol, max_sweeps, rank_cap, log=None, local="elim", kick=2, seed=0):
    """Block-AMEn sweeps (alternating directions) for the Newton system.
    W is a BlockTT warm start whose block core sits at position 0.
    Returns (W, info).  Stopping: the largest relative local residual of the
    incoming iterate over one sweep is below tol (reading: the local
    rounded-system test of Lemma 1)."""
    d = W.d
    L = sysm.L
    Lp = L + 1
    # right-orthogonalise the frame with the block at 0 and build right envs
    envs = Envs(sysm, W)
    for k in range(d - 1, 0, -1):
        envs.update_right(W, k)
    info = dict(sweeps=0, max_res=[], ranks=None)
    tol_svd = tol / math.sqrt(d)
    rng = np.random.default_rng(seed)
    direction = +1
    for sweep in range(max_sweeps):
        max_res = 0.0
        order = range(d) if direction > 0 else range(d - 1, -1, -1)
        for k in order:
            assert W.pos == k
            r, s = W.blk.shape[1], W.blk.shape[3]
            p = r * 4 * s
            K, f, parts = local_system(envs, k, r, s)
            x0 = W.blk[:L].reshape(-1)
            nf = np.linalg.norm(f)
            res0 = np.linalg.norm(K @ x0 - f) / (nf if nf > 0 else 1.0)
            max_res = max(max_res, res0)
            if local == "elim" and not sysm.ineq:
                sol, dz = local_block_elimination(envs, k, r, s)
            else:
                sol = np.linalg.solve(K, f)
                dz = _dz_local(sysm, parts, sol, p)
            blk = np.concatenate([sol, dz]).reshape(Lp, r, 4, s)
            wts = _weights(blk)
            if direction > 0 and k < d - 1:
                U, coef = _split_left(blk, tol_svd, rank_cap, wts, kick, rng)
                W.cores[k] = U
                nxt = W.cores[k + 1]
                W.blk = np.einsum("rls,sit->lrit", coef, nxt)
                W.cores[k + 1] = None
                W.pos = k + 1
                envs.update_left(W, k)
            elif direction < 0 and k > 0:
                V, coef = _split_right(blk, tol_svd, rank_cap, wts, kick, rng)
                W.cores[k] = V
                prv = W.cores[k - 1]
                W.blk = np.einsum("qia,alr->lqir", prv, coef)
                W.cores[k - 1] = None
                W.pos = k - 1
                envs.update_right(W, k)
            else:
                W.blk = blk
        info["sweeps"] += 1
        info["max_res"].append(max_res)
        if log:
            log(f"    amen sweep {sweep} dir {direction:+d} max_res {max_res:.2e} ranks {W.ranks()}")
        direction = -direction
        if max_res < tol and sweep >= 1:
            break
    # leave the block at position 0 for the next warm start
    if W.pos != 0:
        envs_dummy = None
        while W.pos > 0:
            k = W.pos
            wts = _weights(W.blk)
            V, coef = _split_right(W.blk, 0.0, 1 << 30, wts)
            W.cores[k] = V
            W.blk = np.einsum("qia,alr->lqir", W.cores[k - 1], coef)
            W.cores[k - 1] = None
            W.pos = k - 1
    info["ranks"] = W.ranks()
    return W, info


# ----------------------------------------------------------------------------
# the IPM
# ----------------------------------------------------------------------------

def _dense_mat(v):
    n = int(round(math.sqrt(4 ** len(v))))
    return tt.full_mat(tt.unvec_tt(v))


def _max_step_dense(M, dM):
    from .sdp_dense import max_step
    Md = _dense_mat(M)
    dMd = _dense_mat(dM)
    return max_step(0.5 * (Md + Md.T), 0.5 * (dMd + dMd.T))


def _round_shift(v, tol, shift_vec, cap):
    """Cor. 1: round at delta / (1 + ||S||_F), add zeta S; keep unrounded if the
    rank does not drop (and the cap is not exceeded)."""
    nS = tt.norm(shift_vec) if shift_vec is not None else 0.0
    r0 = max(tt.ranks(v))
    vt, zeta = tt.round_tt(v, tol / (1.0 + nS), "abs", cap)
    if max(tt.ranks(vt)) >= r0 and r0 <= cap:
        return v, 0.0
    if shift_vec is not None and zeta > 0:
        vt = tt.add([vt, shift_vec], [1.0, zeta])
    return vt, zeta


def _round_op_shift(L, tol):
    d = len(L)
    I16 = tt.rank1_mat([np.eye(4)] * d)
    nS = float(2 ** d)                      # ||I kron I||_F over 4^d entries
    Lt, zeta = tt.round_tt(L, tol / (1.0 + nS), "abs")
    if max(tt.ranks(Lt)) >= max(tt.ranks(L)):
        return L
    return tt.add([Lt, I16], [1.0, zeta]) if zeta > 0 else Lt


def initial_point(prob):
    """Sec. 5.1: X = Z = lambda* I, Y = 0; with inequalities
    X = lambda* I + (alpha_p / 10) A_ineq(J), T = lambda*_ineq A_ineq(J).
    reading: alpha_p = lambda* / |lambda_min(A_G)| (= lambda* for A_G = J - I)."""
    d = prob["d"]
    lam = prob["lam0"]
    Iv = _ivec(d)
    X = tt.scale(Iv, lam)
    Z = tt.scale(Iv, lam)
    Y = tt.scale(Iv, 0.0)
    T = None
    if "Aineq" in prob:
        J = tt.rank1_vec([np.ones(4)] * d)
        AJ = tt.matvec(prob["Aineq"], J)
        alpha_p = lam / 1.0
        X = tt.add([X, AJ], [1.0, alpha_p / 10.0])
        T = tt.scale(AJ, 1e-3)
    return X, Y, Z, T


def solve(prob, rank_cap=16, eps_gap=1e-4, max_iter=40, eta0=1e-3, delta=1e-4, Cmu=2.0,
          n_xz=3, tau=0.95, amen_sweeps=6, log=None, stop_gap=None, delta_final=None,
          sigma_guard=False, local="elim"):
    """Reference TT-IPM.  Returns a dict with the objective history and the
    final iterates.  stop_gap (default eps_gap) ends the run; the time-to-gap
    mark uses eps_gap with eps_p = eps_d = 2 eps_gap (Sec. 5.1)."""
    t_start = time.perf_counter()
    d, n = prob["d"], prob["n"]
    X, Y, Z, T = initial_point(prob)
    Iv = _ivec(d)
    normB = tt.norm(prob["Beq"])
    normC = tt.norm(prob["C"])
    eta = eta0
    stop_gap = eps_gap if stop_gap is None else stop_gap
    hist = []
    W = None
    q = prob.get("q", 0)
    t_gap = None
    status = "max_iter"
    for it in range(max_iter):
        # --- residuals and measures (Sec. 3.5) ---
        mu = tt.dot(X, Z) / (n + q)
        Rd_t = tt.add([Z, prob["C"], tt.matvec(prob["AeqT"], Y)], [1.0, 1.0, -1.0])
        Rp_t = tt.add([prob["Beq"], tt.matvec(prob["Aeq"], X)], [1.0, -1.0])
        pobj = tt.dot(prob["C"], X)
        dobj = tt.dot(prob["Beq"], Y)
        eps_p = tt.norm(Rp_t) / (1 + normB)
        eps_d = tt.norm(Rd_t) / (1 + normC)
        gap = abs(pobj - dobj) / (1 + abs(pobj) + abs(dobj))
        rec = dict(it=it, mu=mu, pobj=pobj, dobj=dobj, eps_p=eps_p, eps_d=eps_d, gap=gap,
                   rX=max(tt.ranks(X)), rY=max(tt.ranks(Y)), rZ=max(tt.ranks(Z)), eta=eta,
                   t=time.perf_counter() - t_start)
        hist.append(rec)
        if log:
            log(f"it {it:2d} mu {mu:.2e} pobj {pobj:+.8e} dobj {dobj:+.8e} gap {gap:.2e} "
                f"ep {eps_p:.1e} ed {eps_d:.1e} ranks X{rec['rX']} Y{rec['rY']} Z{rec['rZ']}")
        if t_gap is None and gap <= eps_gap and eps_p <= 2 * eps_gap and eps_d <= 2 * eps_gap:
            t_gap = rec["t"]
        if gap <= stop_gap and eps_p <= 2 * stop_gap and eps_d <= 2 * stop_gap:
            status = "converged"
            break
        direction = "xz" if it < n_xz else "aho"
        coef = 1.0 if direction == "xz" else 2.0
        LZ, LX = L_ops(X, Z, direction)
        tolp = eta * (1 + normB) / 10
        told = eta * (1 + normC) / 10
        # reading: the operators are rounded with the Cor. 1 shift (S = I kron I) so
        # that L_Z, L_X stay positive definite when Z, X approach singularity
        LZ = _round_op_shift(LZ, told)
        LX = _round_op_shift(LX, tolp)
        ops = dict(Aeq=prob["Aeq"], AeqT=prob["AeqT"], KY=prob["KY"], LZ=LZ, LX=LX)
        rd = [(1.0, None, Z), (1.0, None, prob["C"]), (-1.0, "AeqT", Y)]
        rp = [(1.0, None, prob["Beq"]), (-1.0, "Aeq", X)]
        if W is None:
            cores = [G.copy() / np.linalg.norm(G) for G in Iv]
            blk = np.zeros((3, 1, 4, 1))
            W = BlockTT(cores, 0, blk)
            W.cores[0] = None
        amen_tol = max(eta / 2, 1e-12)
        # --- predictor (affine, target mu = 0) ---
        rc_aff = [(1.0, "LZ", X)]
        sysm = NewtonSystem(prob, ops, rd, rp, rc_aff)
        W, info_p = amen_solve(sysm, W, amen_tol, amen_sweeps, rank_cap, local=local)
        dX, dY, dZ = W.component(0), W.component(1), W.component(2)
        ap = min(1.0, _max_step_dense(X, dX))
        ad = min(1.0, _max_step_dense(Z, dZ))
        Xa = tt.add([X, dX], [1.0, ap])
        Za = tt.add([Z, dZ], [1.0, ad])
        mu_aff = tt.dot(Xa, Za) / (n + q)
        sigma = (mu_aff / mu) ** 3
        if sigma_guard and hist and "ap" in hist[-1]:
            # reading: after a short step (lost centrality) centre more strongly
            amin = min(hist[-1]["ap"], hist[-1]["ad"])
            if amin < 0.05:
                sigma = max(sigma, 0.7)
            elif amin < 0.2:
                sigma = max(sigma, 0.3)
        # --- corrector with the second-order term L_{dZ_aff} vec dX_aff ---
        Id = identity_mat_tt(d)
        dZm = tt.unvec_tt(dZ)
        if direction == "aho":
            LdZ = tt.add([tt.kron(Id, dZm), tt.kron(dZm, Id)], [1.0, 1.0])
        else:
            LdZ = tt.kron(dZm, Id)
        ops_c = dict(ops)
        ops_c["LdZ"] = LdZ
        rc = [(1.0, "LZ", X), (1.0, "LdZ", dX), (-coef * sigma * mu, None, Iv)]
        sysm_c = NewtonSystem(prob, ops_c, rd, rp, rc)
        W, info_c = amen_solve(sysm_c, W, amen_tol, amen_sweeps, rank_cap, local=local)
        dX, dY, dZ = W.component(0), W.component(1), W.component(2)
        ap = min(1.0, tau * _max_step_dense(X, dX))
        ad = min(1.0, tau * _max_step_dense(Z, dZ))
        # --- update and rounding with spectral shift (Cor. 1) ---
        X, zx = _round_shift(tt.add([X, dX], [1.0, ap]), tolp, Iv, 4 * rank_cap)
        Y, _ = _round_shift(tt.add([Y, dY], [1.0, ad]), told, None, 4 * rank_cap)
        Z, zz = _round_shift(tt.add([Z, dZ], [1.0, ad]), told, Iv, 4 * rank_cap)
        rec.update(ap=ap, ad=ad, sigma=sigma, sweeps=(info_p["sweeps"], info_c["sweeps"]),
                   rW=max(info_c["ranks"]), direction=direction)
        if log:
            log(f"     {direction} sigma {sigma:.2e} ap {ap:.3f} ad {ad:.3f} sweeps {rec['sweeps']} rW {rec['rW']}")
        eta = max(min(eta, Cmu * mu), delta)
    return dict(status=status, hist=hist, X=X, Y=Y, Z=Z, T=T, time_to_gap=t_gap,
                pobj=hist[-1]["pobj"], dobj=hist[-1]["dobj"], gap=hist[-1]["gap"])
