"""GPU TT-IPM against the oracle.

* Newton step (a1-a6 together): at full TT rank the block-AMEn solve is the
  dense Newton solve, so the corrector direction of one ttipm_step equals the
  dense Mehrotra corrector of eq. (tt-kkt-newton-system) built by the oracle
  (relative error <= 1e-8; the dense system at the initial point is well
  conditioned, so this bounds the whole chain of contractions, local solves,
  SVD moves and step lengths).
* Whole solves: objective within 1e-6 (relative) of closed-form SDP values and
  of the dense IPM oracle; the time-to-gap mark is reached.
"""
import math

import numpy as np
import pytest

import instances as I
from oracle import kkt, problems as OP, sdp_dense as S, tt as ott

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2509_11890_amd as P
    return P


def _perm(d):
    """index map: vec_TT position of entry (r, c) of a 2^d x 2^d matrix."""
    n = 2 ** d
    idx = np.zeros((n, n), dtype=np.int64)
    for r in range(n):
        for c in range(n):
            v = 0
            for k in range(d):
                v = v * 4 + 2 * ((r >> (d - 1 - k)) & 1) + ((c >> (d - 1 - k)) & 1)
            idx[r, c] = v
    return idx


def _mat(v, idx):
    return v[idx]


def _vec(M, idx):
    out = np.zeros(M.size)
    out[idx.reshape(-1)] = M.reshape(-1)
    return out


def _dense_corrector(prob, direction):
    """Oracle Mehrotra step at the initial point: predictor, Thm. 1 steps, sigma,
    corrector with the second-order term (dense)."""
    d = prob["d"]
    n = 2 ** d
    idx = _perm(d)
    lam = prob["lam0"]
    Xt = ott.scale(OP._const_vec(OP._I4, d), lam)
    Zt = ott.scale(OP._const_vec(OP._I4, d), lam)
    Yt = ott.scale(OP._const_vec(OP._I4, d), 0.0)
    x, z = ott.full(Xt), ott.full(Zt)
    mu = x @ z / n
    dX, dY, _, dZ = kkt.newton_dense(prob, Xt, Yt, Zt, None, mu, direction, sigma_mu=0.0)
    X, Z = _mat(x, idx), _mat(z, idx)
    sym = lambda A: 0.5 * (A + A.T)
    ap = min(1.0, S.max_step(sym(X), sym(_mat(dX, idx))))
    ad = min(1.0, S.max_step(sym(Z), sym(_mat(dZ, idx))))
    mu_aff = (x + ap * dX) @ (z + ad * dZ) / n
    sigma = (mu_aff / mu) ** 3
    DX, DZ = _mat(dX, idx), _mat(dZ, idx)
    coef = 2.0 if direction == "aho" else 1.0
    second = DZ @ DX + DX @ DZ if direction == "aho" else DZ @ DX
    _, _, _, Rc = kkt.residuals_dense(prob, Xt, Yt, Zt, None, mu, direction, sigma_mu=sigma * mu)
    Rc = Rc + _vec(second, idx)
    return kkt.newton_dense(prob, Xt, Yt, Zt, None, mu, direction, Rc_override=Rc)


@pytest.mark.parametrize("kind,graph", [("maxcut", I.complete(3)), ("maxcut", I.odd_cycle_plus_isolated(3)),
                                        ("theta", I.c5_plus_3k1()), ("maxcut", I.grid_4x8())],
                         ids=["K8", "C7+K1", "C5+3K1", "grid4x8-d5"])
@pytest.mark.parametrize("direction", ["xz", "aho"])
def test_full_rank_step_equals_dense_newton(kind, graph, direction):
    """At full TT rank the corrector direction of one ttipm_step is the dense
    Mehrotra corrector: every entry of dX, dY, dZ within 1e-10 of the largest
    entry of the dense solution (d = 3 and the 4 x 8 grid at d = 5, whose
    middle local system has 2 x 4096 unknowns)."""
    P = _lib()
    prob = OP.maxcut(graph.cores) if kind == "maxcut" else OP.theta(graph.cores)
    ref = _dense_corrector(prob, direction)
    kid = P.TTIPM_MAXCUT if kind == "maxcut" else P.TTIPM_THETA
    pr = P.Problem(kid, graph.cores)
    prm = P.Params(eta0=1e-13, delta=1e-13, rank_cap=64, iter_rank_cap=256, amen_sweeps=8,
                   n_xz=3 if direction == "xz" else 0, eig_rank=64, eig_sweeps=3, direct_max=8192)
    st = P.State(pr, prm)
    P.ttipm_step(pr, st, prm)
    for comp, r in zip("xyz", (ref[0], ref[1], ref[3])):
        got = ott.full(st.export(comp))
        err = np.max(np.abs(got - r)) / max(np.max(np.abs(r)), 1e-300)
        assert err < 1e-10, (comp, err)


CLOSED = [
    ("K16", "maxcut", lambda: I.complete(4), 64.0),
    ("C7+K1", "maxcut", lambda: I.odd_cycle_plus_isolated(3), 3.5 * (1 + math.cos(math.pi / 7))),
    ("Q5-maxcut", "maxcut", lambda: I.hypercube(5), 80.0),
    ("theta-Q5", "theta", lambda: I.hypercube(5), 16.0),
    ("theta-C5+3K1", "theta", lambda: I.c5_plus_3k1(), 3 + math.sqrt(5)),
    ("grid-4x8", "maxcut", lambda: I.grid_4x8(), 52.0),
    ("K32", "maxcut", lambda: I.complete(5), 256.0),
]

# n = 1024 members of the closed-form suite: the 1e-4 time-to-gap mark (rel_gap <= 1e-4,
# eps_p, eps_d <= 2e-4) at TT ranks <= 8.  rel_gap is normalised by 1 + |p| + |d| (about twice
# the value), so at the mark each objective lies within about 2e-4 of the value (relative).
CLOSED_D10 = [
    ("K1024", lambda: I.complete(10), 1024.0 ** 2 / 4),
    ("Q10-maxcut", lambda: I.hypercube(10), 10 * 512.0),
]


@pytest.mark.parametrize("name,make,value", CLOSED_D10, ids=[c[0] for c in CLOSED_D10])
def test_d10_maxcut_reaches_gap_mark(name, make, value):
    P = _lib()
    g = make()
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=8, iter_rank_cap=8, stop_gap=1e-4, max_iter=60)
    st = P.State(pr, prm)
    res, log = P.ttipm_solve(pr, st, prm)
    print(name, res)
    assert res["status"] == P.TT_OK and res["time_to_gap"] > 0
    assert abs(res["pobj"] - value) / (1 + value) < 2.5e-4
    assert abs(res["dobj"] - value) / (1 + value) < 2.5e-4


@pytest.mark.parametrize("name,kind,make,value", CLOSED, ids=[c[0] for c in CLOSED])
def test_solve_matches_closed_form(name, kind, make, value):
    P = _lib()
    g = make()
    pr = P.Problem(P.TTIPM_MAXCUT if kind == "maxcut" else P.TTIPM_THETA, g.cores)
    # the grid instance is run at its configuration: TT ranks <= 8 for the iterates and the Newton frame
    caps = dict(rank_cap=8, iter_rank_cap=8, max_iter=100) if name == "grid-4x8" else \
        dict(rank_cap=8 if g.d >= 5 else 16, max_iter=100)
    prm = P.Params(stop_gap=3e-7, delta=1e-10, **caps)
    st = P.State(pr, prm)
    res, log = P.ttipm_solve(pr, st, prm)
    print(name, res)
    assert res["time_to_gap"] > 0                         # gap 1e-4 with eps_p, eps_d <= 2e-4
    assert abs(res["pobj"] - value) / (1 + value) < 1e-6
    assert abs(res["dobj"] - value) / (1 + value) < 1e-6


@pytest.mark.parametrize("enabled", [0, 1])
def test_aho_to_xz_fallback_is_taken_and_logged(enabled):
    """A frame capped at rank 1 with a single sweep cannot meet the AHO residual
    target, so with the fallback on AHO iterations are redone with XZ (and
    logged); with it off none is."""
    P = _lib()
    g = I.complete(4)
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=1, amen_sweeps=1, n_xz=1, max_iter=6, xz_fallback=enabled)
    st = P.State(pr, prm)
    res, log = P.ttipm_solve(pr, st, prm)
    aho_iters = [l for l in log if l["iter"] >= 1]
    assert aho_iters and all(np.isfinite(l["pobj"]) for l in log)
    flags = [l["xz_fallback"] for l in aho_iters]
    assert (any(flags) if enabled else not any(flags)), flags


def test_c1_grid_matches_dense_oracle():
    """Config 1 (4x8 grid, d = 5, TT ranks <= 8, FP64): objective vs the dense IPM."""
    P = _lib()
    g = I.grid_4x8()
    dense = S.solve(OP.maxcut_dense(g.dense))
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=8, iter_rank_cap=8, stop_gap=3e-7, delta=1e-10, max_iter=100)
    st = P.State(pr, prm)
    res, log = P.ttipm_solve(pr, st, prm)
    assert max(l["rank_x"] for l in log) <= 9          # rank 8 plus the rank-1 shift of Cor. 1
    assert abs(res["pobj"] - dense["pobj"]) / (1 + abs(dense["pobj"])) < 1e-6


def _tt_vector_exact(v, d):
    """Exact TT (mode 2) of a length-2^d vector by successive SVDs (input data)."""
    cores, r, C = [], 1, np.asarray(v, dtype=np.float64).reshape(1, -1)
    for k in range(d - 1):
        C = C.reshape(r * 2, -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = max(1, int(np.sum(s > 1e-14 * max(s[0], 1e-300))))
        cores.append(U[:, :rk].reshape(r, 2, rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, 2, 1))
    return cores


@pytest.mark.parametrize("combine", [1, 0], ids=["combined", "separate"])
@pytest.mark.parametrize("d,terms,seed", [(3, 2, 7), (4, 2, 3)])
def test_cc_matches_dense_oracle(d, terms, seed, combine):
    """Correlation clustering (inequality constraints X_uv >= 0 on all pairs,
    mirrored multipliers T, K_T; Sec. 4.3) against the dense IPM oracle, with
    the multiplier updates in one combined block dL (disjoint masks, Sec. 3.5)
    and as separate dY, dT blocks."""
    P = _lib()
    g = I.signed_kron(d, terms, seed)
    W = g.dense
    dense = S.solve(OP.cc_dense(W))
    negdeg = np.maximum(-W, 0.0).sum(axis=1)
    pr = P.Problem(P.TTIPM_CC, g.cores, _tt_vector_exact(negdeg, d))
    prm = P.Params(rank_cap=64, stop_gap=3e-7, delta=1e-10, max_iter=80, combine_multipliers=combine)
    st = P.State(pr, prm)
    res, log = P.ttipm_solve(pr, st, prm)
    print("cc", d, res, dense["pobj"])
    assert res["time_to_gap"] > 0
    assert abs(res["pobj"] - dense["pobj"]) / (1 + abs(dense["pobj"])) < 1e-6


def _ratio(v, dv, mask):
    """largest alpha with v + alpha dv >= 0 on the mask (inf if unbounded)."""
    sel = (mask > 0.5) & (dv < 0)
    return np.inf if not np.any(sel) else float(np.min(np.maximum(v[sel], 0.0) / -dv[sel]))


def _dense_corrector_cc(prob, X0, Y0, Z0, T0, direction):
    """Oracle Mehrotra step for the correlation-clustering system (slack and
    multiplier ratio tests, mu with <T, s>, R_t second-order term)."""
    d = prob["d"]
    n = 2 ** d
    idx = _perm(d)
    f = ott.full
    x, z, t = f(X0), f(Z0), f(T0)
    Ai = ott.full_mat(prob["Aineq"])
    sg = prob["sense"]
    mask = f(kkt.one_T(prob))
    q = int(round(mask.sum()))
    slack = sg * (f(prob["Bineq"]) - Ai @ x)
    mu = (x @ z + t @ slack) / (n + q)
    dX, dY, dT, dZ = kkt.newton_dense(prob, X0, Y0, Z0, T0, mu, direction, sigma_mu=0.0)
    sym = lambda A: 0.5 * (A + A.T)
    X, Z = _mat(x, idx), _mat(z, idx)
    ds = -sg * (Ai @ dX)
    ap = min(1.0, S.max_step(sym(X), sym(_mat(dX, idx))), _ratio(slack, ds, mask))
    ad = min(1.0, S.max_step(sym(Z), sym(_mat(dZ, idx))), _ratio(t, dT, mask))
    mu_aff = ((x + ap * dX) @ (z + ad * dZ) + (t + ad * dT) @ (slack + ap * ds)) / (n + q)
    sigma = (mu_aff / mu) ** 3
    DX, DZ = _mat(dX, idx), _mat(dZ, idx)
    coef = 2.0 if direction == "aho" else 1.0
    second = DZ @ DX + DX @ DZ if direction == "aho" else DZ @ DX
    _, _, Rt, Rc = kkt.residuals_dense(prob, X0, Y0, Z0, T0, mu, direction, sigma_mu=sigma * mu)
    return kkt.newton_dense(prob, X0, Y0, Z0, T0, mu, direction, Rc_override=Rc + _vec(second, idx),
                            Rt_override=Rt + dT * ds)


@pytest.mark.parametrize("combine", [1, 0], ids=["combined", "separate"])
@pytest.mark.parametrize("direction", ["aho"])
def test_full_rank_cc_step_equals_dense_newton(direction, combine):
    """Correlation clustering at full TT rank: the corrector direction of one
    ttipm_step (block AMEn with the inequality block row, slack and multiplier
    ratio tests, mu with <T, s>, R_t second-order term) equals the dense
    Mehrotra corrector of the oracle."""
    P = _lib()
    d = 3
    g = I.signed_kron(d, 2, 7)
    negdeg = np.maximum(-g.dense, 0.0).sum(axis=1)
    nd = _tt_vector_exact(negdeg, d)
    prob = OP.cc(g.cores, nd)
    pr = P.Problem(P.TTIPM_CC, g.cores, nd)
    prm = P.Params(eta0=1e-13, delta=1e-13, rank_cap=64, iter_rank_cap=256, amen_sweeps=8,
                   n_xz=3 if direction == "xz" else 0, eig_rank=64, eig_sweeps=3, combine_multipliers=combine)
    st = P.State(pr, prm)
    # initial point of Sec. 5.1 with inequalities (reading: alpha_p = lambda* = 2 for A_G = J - I,
    # lambda*_ineq = 1e-3): X = 2 I + 0.2 (J - I), Z = 2 I, Y = 0, T = 1e-3 (J - I)
    Iv = ott.rank1_vec([np.array([1.0, 0.0, 0.0, 1.0])] * d)
    Jv = ott.rank1_vec([np.ones(4)] * d)
    JmI = ott.add([Jv, Iv], [1.0, -1.0])
    X0 = ott.add([Iv, JmI], [2.0, 0.2])
    Z0 = ott.scale(Iv, 2.0)
    Y0 = ott.scale(Iv, 0.0)
    T0 = ott.scale(JmI, 1e-3)
    ref = _dense_corrector_cc(prob, X0, Y0, Z0, T0, direction)
    P.ttipm_step(pr, st, prm)
    for comp, r in zip("xytz", ref):
        got = ott.full(st.export(comp))
        err = np.max(np.abs(got - r)) / max(np.max(np.abs(r)), 1e-300)
        assert err < 1e-10, (comp, err)


def test_checkpoint_resume_through_state_import():
    """Checkpoint / resume: iterates exported after a few steps and imported
    into a fresh state are the same TTs (bit for bit), give the same measures at
    entry of the next step, and the resumed solve reaches the closed-form value
    (MaxCut on K_32: n^2/4 = 256).  Malformed imports are rejected."""
    P = _lib()
    g = I.complete(5)
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=8, stop_gap=3e-7, delta=1e-10, max_iter=60)
    a = P.State(pr, prm)
    for _ in range(4):
        P.ttipm_step(pr, a, prm)
    saved = {w: a.export(w) for w in "XYZ"}
    b = P.State(pr, prm)
    for w, cores in saved.items():
        b.import_(w, cores)
        back = b.export(w)
        assert [G.shape for G in back] == [G.shape for G in cores]
        assert all(np.array_equal(G, H) for G, H in zip(back, cores))
    ia, ib = P.ttipm_step(pr, a, prm), P.ttipm_step(pr, b, prm)
    for k in ("mu", "pobj", "dobj", "eps_p", "eps_d"):
        assert abs(ia[k] - ib[k]) <= 1e-12 * (1 + abs(ia[k])), (k, ia[k], ib[k])

    res, _ = P.ttipm_solve(pr, b, prm)
    assert abs(res["pobj"] - 256.0) / 257.0 < 1e-6 and abs(res["dobj"] - 256.0) / 257.0 < 1e-6

    bad = [G.copy() for G in saved["X"]]
    with pytest.raises(P.TTError):
        b.import_("Q", bad)
    with pytest.raises(P.TTError):                     # inner rank mismatch between neighbours
        b.import_("X", bad[:-1] + [np.zeros((bad[-1].shape[0] + 1, 4, 1))])


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_krylov_local_solves_reach_gap_mark(precision):
    """Local systems above 64 unknowns through restarted GMRES with block
    Jacobi: in FP64 every Krylov product runs the grouped stage products of
    the local KKT operator, in mixed precision the per-operator BF16 products
    with FP64 refinement.  The 4x8 grid (value 52, TT ranks <= 8) reaches the
    1e-4 gap mark with both objectives within 2.5e-4 of the value."""
    P = _lib()
    g = I.grid_4x8()
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=8, iter_rank_cap=8, stop_gap=1e-4, eps_gap=1e-4, max_iter=100, direct_max=64,
                   precond=P.TT_PREC_BJACOBI, gmres_restart=40, gmres_maxit=800,
                   precision=P.TTIPM_F64 if precision == "f64" else P.TTIPM_MIXED)
    st = P.State(pr, prm)
    res, log = P.ttipm_solve(pr, st, prm)
    print(precision, res, sum(l["krylov_iters"] for l in log))
    assert sum(l["krylov_iters"] for l in log) > 0
    assert res["status"] == P.TT_OK and res["time_to_gap"] > 0
    assert abs(res["pobj"] - 52.0) / 53.0 < 2.5e-4 and abs(res["dobj"] - 52.0) / 53.0 < 2.5e-4


def test_solve_is_reproducible_run_to_run():
    """The primal and dual phases run on two streams and every reduction has a
    fixed order, so two solves of one instance from fresh states agree bit for
    bit, iteration by iteration."""
    P = _lib()
    g = I.grid_4x8()
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=8, iter_rank_cap=8, stop_gap=1e-4, max_iter=40, direct_max=64,
                   precond=P.TT_PREC_BJACOBI)
    runs = []
    for _ in range(2):
        st = P.State(pr, prm)
        res, log = P.ttipm_solve(pr, st, prm)
        runs.append([(l["pobj"], l["dobj"], l["alpha_p"], l["alpha_d"], l["krylov_iters"]) for l in log])
    assert len(runs[0]) > 3 and runs[0] == runs[1]


def _generic_from_oracle(P, prob):
    kw = dict(C_=prob["C"], Aeq=prob["Aeq"], AeqT=prob["AeqT"], Beq=prob["Beq"], KY=prob["KY"],
              lam0=prob["lam0"])
    if "Aineq" in prob:
        kw.update(Aineq=prob["Aineq"], AineqT=prob["AineqT"], Bineq=prob["Bineq"], KT=prob["KT"],
                  ineq_sense=int(prob["sense"]), q=float(prob["q"]), x0_ineq=prob["lam0"] / 10.0, t0_ineq=1e-3)
    return P.Problem.generic(**kw)


@pytest.mark.parametrize("which", ["grid_maxcut", "c5_3k1_theta", "cc_d3"])
def test_generic_problem_matches_built_kind(which):
    """The same SDP given as TTIPM_GENERIC (the oracle's Sec. 4 encodings passed
    as C, A_eq, A_eq^T, B_eq, K_Y [, A_ineq, A_ineq^T, B_ineq, K_T]) and built
    by the library from the graph: the solves take the same iterations and end
    at the same iterate (the operators agree to rounding, so the trajectories
    agree to far below the stopping tolerances)."""
    P = _lib()
    if which == "grid_maxcut":
        g = I.grid_4x8()
        kind, prob, nd, caps = P.TTIPM_MAXCUT, OP.maxcut(g.cores), None, dict(rank_cap=8, iter_rank_cap=8)
    elif which == "c5_3k1_theta":
        g = I.c5_plus_3k1()
        kind, prob, nd, caps = P.TTIPM_THETA, OP.theta(g.cores), None, dict(rank_cap=16)
    else:
        g = I.signed_kron(3, 2, 7)
        nd = I.negdeg_cores(g)
        kind, prob, caps = P.TTIPM_CC, OP.cc(g.cores, nd), dict(rank_cap=64)
    built = P.Problem(kind, g.cores, nd)
    gen = _generic_from_oracle(P, prob)
    prm = P.Params(stop_gap=1e-6, delta=1e-8, max_iter=60, **caps)
    out = []
    for pr in (built, gen):
        st = P.State(pr, prm)
        res, log = P.ttipm_solve(pr, st, prm)
        X = ott.full(st.export("X"))
        out.append((res, X))
    (r0, X0), (r1, X1) = out
    print(which, r0, r1)
    assert r0["iterations"] == r1["iterations"]
    assert abs(r0["pobj"] - r1["pobj"]) <= 1e-8 * (1 + abs(r0["pobj"]))
    assert abs(r0["dobj"] - r1["dobj"]) <= 1e-8 * (1 + abs(r0["dobj"]))
    assert np.linalg.norm(X0 - X1) <= 1e-7 * np.linalg.norm(X0)


def _merit(l):
    return l["norm_rp"] + l["norm_rd"] + abs(l["xz"])


@pytest.mark.parametrize("d,seed", [(4, 3), (3, 7)])
def test_finishing_phase_reaches_absolute_targets_cc(d, seed):
    """Finishing phase (Sec. 3.5, relaxing the PD barrier): on the
    correlation-clustering instances at full TT rank, the solve continues past
    the relative criteria (1e-4) to the absolute targets ||R_p||, ||R_d||,
    <X, Z> < 1e-6 under merit-based acceptance.  The merit of the entry
    iterates never rises, every finishing iterate still meets the relative
    criteria, and both objectives land within 1e-6 of the dense IPM oracle;
    without the phase the same run stops with ||R_d|| far above the target."""
    P = _lib()
    g = I.signed_kron(d, 2, seed)
    dense = S.solve(OP.cc_dense(g.dense))
    pr = P.Problem(P.TTIPM_CC, g.cores, _tt_vector_exact(np.maximum(-g.dense, 0.0).sum(axis=1), d))
    runs = {}
    for fin in (0, 1):
        prm = P.Params(rank_cap=64, stop_gap=1e-4, eps_gap=1e-4, max_iter=60, finish=fin, finish_abs=1e-6)
        runs[fin] = P.ttipm_solve(pr, P.State(pr, prm), prm)
    res0, _ = runs[0]
    res, log = runs[1]
    print("finish", d, {k: res[k] for k in ("iterations", "finish_iterations", "norm_rp", "norm_rd", "xz",
                                           "pobj", "dobj")}, dense["pobj"])
    assert res0["status"] == 0 and res0["absolute_met"] == 0 and res0["finish_iterations"] == 0
    assert res["status"] == 0 and res["absolute_met"] == 1 and res["finish_iterations"] > 0
    assert res["norm_rp"] < 1e-6 and res["norm_rd"] < 1e-6 and res["xz"] < 1e-6
    for key in ("pobj", "dobj"):
        assert abs(res[key] - dense["pobj"]) / (1 + abs(dense["pobj"])) < 1e-6
    fin = [l for l in log if l["finishing"]]
    assert fin
    for a, b in zip(fin, fin[1:]):
        assert _merit(b) <= _merit(a) * (1 + 1e-12)
        if a["finish_rejected"]:
            assert _merit(b) == _merit(a)
    for l in fin:
        assert l["rel_gap"] <= 1e-4 and l["eps_p"] <= 2e-4 and l["eps_d"] <= 2e-4


def test_finishing_phase_keeps_relative_criteria_when_capped():
    """With rank caps that keep the absolute targets out of reach (4 x 8 grid
    MaxCut, caps 8/8), the finishing phase stops on its own (rejections or
    max_iter), and the result still meets the relative criteria with an
    objective no further from the closed form (52) than the relative
    criteria allow."""
    P = _lib()
    g = I.grid_4x8()
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    prm = P.Params(rank_cap=8, iter_rank_cap=8, stop_gap=1e-4, eps_gap=1e-4, max_iter=40, finish=1)
    res, log = P.ttipm_solve(pr, P.State(pr, prm), prm)
    assert res["status"] == 0 and res["finish_iterations"] > 0
    assert res["rel_gap"] <= 1e-4 and res["eps_p"] <= 2e-4 and res["eps_d"] <= 2e-4
    assert abs(res["pobj"] - 52.0) / 53.0 < 3e-4
    fin = [l for l in log if l["finishing"]]
    for a, b in zip(fin, fin[1:]):
        assert _merit(b) <= _merit(a) * (1 + 1e-12)


def test_global_stop_saves_half_sweeps_on_capped_grid():
    """The global-residual stopping rule of capped AMEn solves: on the 4 x 8
    grid at caps 8/8 the solve still reaches the gap mark with the objective
    within the mark's accuracy of 52, with fewer AMEn half-sweeps than the
    local rule alone, and every iteration reports the global ratio it
    stopped on."""
    P = _lib()
    g = I.grid_4x8()
    pr = P.Problem(P.TTIPM_MAXCUT, g.cores)
    sweeps = {}
    for flag in (0, 1):
        prm = P.Params(rank_cap=8, iter_rank_cap=8, stop_gap=1e-4, eps_gap=1e-4, max_iter=60, amen_global_stop=flag)
        res, log = P.ttipm_solve(pr, P.State(pr, prm), prm)
        assert res["status"] == 0 and res["time_to_gap"] > 0
        assert abs(res["pobj"] - 52.0) / 53.0 < 3e-4
        sweeps[flag] = sum(l["sweeps_pred"] + l["sweeps_corr"] for l in log) / len(log)
        assert all(l["newton_res"] >= 0.0 for l in log)
    assert sweeps[1] < sweeps[0]
