"""Dense primal-dual interior-point method for the benchmark SDPs (oracle).

Plain FP64 NumPy/LAPACK.  Solves the primal SDP of Sec. 2.2 (Def. "SDP")
    max C . X  s.t.  A_eq(X) = b_eq,  A_ineq(X) >= b_ineq (as slack rows),  X psd
together with its dual (Def. "The Dual SDP"), following Alg. 1 of the paper:
residuals -> Newton direction -> maximal step by Thm. 1 (Cholesky + lambda_max)
-> update.  The Newton direction is the HKM direction with Mehrotra's
predictor-corrector (Sec. 3.5 names Mehrotra's method; the dense oracle uses
the HKM symmetrisation, a standard direction with the same optimum as the AHO
direction the TT method uses).  The optimum value is unique, so only values and
certificates are compared with the TT method.

Internally the problem is put in the textbook min form
    min -C . X  s.t.  A_i . X + g_i^T s = b_i,  X psd, s >= 0,
with s the slacks of the inequality rows (g_i = -e for A_i . X - s_i = b_i).
Constraint families (the Schur complement is formed family by family):
    ("diag",  idx, rhs)      A_i = e_p e_p^T
    ("pair",  (a, b), rhs)   A_i = (e_a e_b^T + e_b e_a^T) / 2
    ("trace", None, rhs)     A_i = I
"""
from __future__ import annotations

import time
import numpy as np
import scipy.linalg as sla


def _fam_size(f, n):
    kind, idx, rhs = f
    if kind == "diag":
        return len(idx)
    if kind == "pair":
        return len(idx[0])
    return 1


def _apply_A(fams, X):
    out = []
    for kind, idx, _ in fams:
        if kind == "diag":
            out.append(X[idx, idx])
        elif kind == "pair":
            a, b = idx
            out.append(0.5 * (X[a, b] + X[b, a]))
        else:
            out.append(np.array([np.trace(X)]))
    return np.concatenate(out) if out else np.zeros(0)


def _apply_AT(fams, y, n):
    M = np.zeros((n, n))
    o = 0
    for f in fams:
        kind, idx, _ = f
        m = _fam_size(f, n)
        yy = y[o:o + m]
        if kind == "diag":
            M[idx, idx] += yy
        elif kind == "pair":
            a, b = idx
            np.add.at(M, (a, b), 0.5 * yy)
            np.add.at(M, (b, a), 0.5 * yy)
        else:
            M += yy[0] * np.eye(n)
        o += m
    return M


def _schur_block(fi, fj, X, W, XW, WX):
    """M_ij = A_i . (X A_j W) for two constraint families."""
    ki, ii, _ = fi
    kj, jj, _ = fj
    if ki == "diag" and kj == "diag":
        return X[np.ix_(ii, jj)] * W[np.ix_(jj, ii)].T
    if ki == "diag" and kj == "pair":
        c, d = jj
        return 0.5 * (X[np.ix_(ii, c)] * W[np.ix_(d, ii)].T + X[np.ix_(ii, d)] * W[np.ix_(c, ii)].T)
    if ki == "pair" and kj == "diag":
        a, b = ii
        return 0.5 * (X[np.ix_(a, jj)] * W[np.ix_(jj, b)].T + X[np.ix_(b, jj)] * W[np.ix_(jj, a)].T)
    if ki == "pair" and kj == "pair":
        a, b = ii
        c, d = jj
        return 0.25 * (X[np.ix_(a, c)] * W[np.ix_(d, b)].T + X[np.ix_(a, d)] * W[np.ix_(c, b)].T
                       + X[np.ix_(b, c)] * W[np.ix_(d, a)].T + X[np.ix_(b, d)] * W[np.ix_(c, a)].T)
    if ki == "trace" and kj == "trace":
        return np.array([[np.trace(XW)]])
    if ki == "trace":
        # I . (X A_j W) = A_j . (W X)
        if kj == "diag":
            return WX[jj, jj][None, :]
        c, d = jj
        return (0.5 * (WX[d, c] + WX[c, d]))[None, :]
    # kj == "trace": A_i . (X W)
    if ki == "diag":
        return XW[ii, ii][:, None]
    a, b = ii
    return (0.5 * (XW[a, b] + XW[b, a]))[:, None]


def _schur(fams, X, W):
    XW, WX = X @ W, W @ X
    n = X.shape[0]
    rows = []
    for fi in fams:
        rows.append(np.hstack([_schur_block(fi, fj, X, W, XW, WX) for fj in fams]))
    return np.vstack(rows)


def max_step(M, dM):
    """Thm. 1: largest alpha with M + alpha dM psd (M pd), via the Cholesky
    factor L of M and lambda_max(-L^{-1} dM L^{-T}); returns inf if dM psd."""
    L = np.linalg.cholesky(M)
    Li = sla.solve_triangular(L, np.eye(M.shape[0]), lower=True)
    B = -Li @ dM @ Li.T
    lam = np.linalg.eigvalsh(0.5 * (B + B.T))[-1]
    return np.inf if lam <= 0 else 1.0 / lam


def _max_step_lp(s, ds):
    neg = ds < 0
    return np.inf if not np.any(neg) else float(np.min(-s[neg] / ds[neg]))


def solve(prob, tol_gap=1e-9, tol_feas=1e-10, max_iter=100, tau=0.95, lam0=None,
          log=None, gap_marks=(1e-4,)):
    """Dense HKM/Mehrotra IPM.  Returns a dict with pobj, dobj, X, y (equality
    multipliers, in the max-form convention Z = A^T y - C - A_ineq^T t), Z,
    iterations and the wall time at which rel_gap first fell below each mark."""
    t0 = time.perf_counter()
    n = prob["n"]
    C = np.asarray(prob["C"], dtype=np.float64)
    eq, ineq = prob["eq"], prob["ineq"]
    fams = list(eq) + list(ineq)
    meq = sum(_fam_size(f, n) for f in eq)
    q = sum(_fam_size(f, n) for f in ineq)
    m = meq + q
    b = np.concatenate([f[2] for f in fams]) if fams else np.zeros(0)
    Cm = -C                                        # min-form objective
    # initial point
    lam = 1.0 if lam0 is None else lam0
    X = lam * np.eye(n)
    S = lam * np.eye(n)
    y = np.zeros(m)
    s = np.ones(q)
    z = np.ones(q)
    marks = {g: None for g in gap_marks}
    hist = []
    status = "max_iter"
    normb, normC = np.linalg.norm(b), np.linalg.norm(C)
    for it in range(max_iter):
        AX = _apply_A(fams, X)
        rp = b - AX
        rp[meq:] += s                              # A_ineq X - s = b_ineq
        Rd = Cm - _apply_AT(fams, y, n) - S
        rz = y[meq:] - z                           # -g^T y - z with g = -e
        pobj = float(np.sum(C * X))
        dobj = float(-(b @ y))
        gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
        pinf = np.linalg.norm(rp) / (1.0 + normb)
        dinf = np.sqrt(np.linalg.norm(Rd) ** 2 + np.linalg.norm(rz) ** 2) / (1.0 + normC)
        hist.append((it, pobj, dobj, gap, pinf, dinf))
        if log:
            log(f"it {it:3d} pobj {pobj:+.10e} dobj {dobj:+.10e} gap {gap:.2e} pinf {pinf:.2e} dinf {dinf:.2e}")
        for g in marks:
            if marks[g] is None and gap <= g and pinf <= 2 * g and dinf <= 2 * g:
                marks[g] = time.perf_counter() - t0
        if gap <= tol_gap and pinf <= tol_feas and dinf <= tol_feas:
            status = "optimal"
            break
        mu = (np.sum(X * S) + s @ z) / (n + q)
        W = np.linalg.inv(S)
        W = 0.5 * (W + W.T)
        M = _schur(fams, X, W)
        if q:
            M[meq:, meq:] += np.diag(s / z)
        M = 0.5 * (M + M.T)
        try:
            cf = sla.cho_factor(M)
            solveM = lambda r: sla.cho_solve(cf, r)
        except np.linalg.LinAlgError:       # M is pd in exact arithmetic; near mu -> 0
            lu = sla.lu_factor(M)           # rounding can break Cholesky, LU still solves
            solveM = lambda r: sla.lu_solve(lu, r)

        def direction(sigma, corrX=None, corrs=None):
            K = sigma * mu * W - X
            if corrX is not None:
                K = K - corrX @ W
            ks = sigma * mu / z - s if q else np.zeros(0)
            if corrs is not None:
                ks = ks - corrs / z
            G = K - X @ Rd @ W
            gs = ks - s * rz / z if q else ks
            rhs = rp - _apply_A(fams, G)
            if q:
                rhs[meq:] += gs                    # -(g gs) with g = -e
            dy = solveM(rhs)
            dS = Rd - _apply_AT(fams, dy, n)
            dX = G + X @ _apply_AT(fams, dy, n) @ W
            dX = 0.5 * (dX + dX.T)
            if q:
                dz = rz + dy[meq:]                 # -g^T dy with g = -e
                ds = gs - s * dy[meq:] / z
            else:
                dz = ds = np.zeros(0)
            return dX, dy, dS, ds, dz

        # predictor
        dX, dy, dS, ds, dz = direction(0.0)
        ap = min(1.0, max_step(X, dX), _max_step_lp(s, ds) if q else np.inf)
        ad = min(1.0, max_step(S, dS), _max_step_lp(z, dz) if q else np.inf)
        mu_aff = (np.sum((X + ap * dX) * (S + ad * dS)) + (s + ap * ds) @ (z + ad * dz)) / (n + q)
        sigma = (mu_aff / mu) ** 3
        # corrector (second-order term dX_aff dS_aff)
        dX, dy, dS, ds, dz = direction(sigma, corrX=dX @ dS, corrs=ds * dz if q else None)
        ap = min(1.0, tau * max_step(X, dX), tau * _max_step_lp(s, ds) if q else np.inf)
        ad = min(1.0, tau * max_step(S, dS), tau * _max_step_lp(z, dz) if q else np.inf)
        X = X + ap * dX
        s = s + ap * ds
        y = y + ad * dy
        S = S + ad * dS
        z = z + ad * dz
        X = 0.5 * (X + X.T)
        S = 0.5 * (S + S.T)
    # max-form multipliers: Z = S, y_max = -y
    return dict(status=status, pobj=pobj, dobj=dobj, gap=gap, pinf=pinf, dinf=dinf, X=X, Z=S,
                y=-y[:meq], t=y[meq:], iterations=len(hist) - 1, hist=hist,
                time=time.perf_counter() - t0, time_to_gap=marks)
