"""Seeded synthetic SDP instances: graph data in tensor-train (TT) matrix form.

This module only *describes graphs*.  It holds none of the interior-point or
TT-solver arithmetic; both the CPU oracle and the HIP library build their own
SDP operators (objective, constraint operators, masks) from what is returned
here.

Conventions (paper, Sec. 2.3, Def. "TT Matrix" and the big-endian remark):
a 2^d x 2^d matrix A is stored as d cores G_k of shape [R_k, 2, 2, R_{k+1}]
(R_1 = R_{d+1} = 1) with A[alpha; beta] = G_1(alpha_1, beta_1) ... G_d(alpha_d,
beta_d), where alpha = sum_k alpha_k 2^(d-k), i.e. core 1 holds the most
significant bit.  Every instance also carries an independently built dense
adjacency matrix (for n <= 4096) so that the TT form can be checked.

Instances (graph families with sizes and seeds):
  grid_4x8              4x8 grid, vertex v = 8 i + j (i = two MSBs), unit weights
  kron_sum_products     sum of T Kronecker products of random symmetric U[0,1]
                        2x2 factors, diagonal removed (MaxCut weights)
  hypercube             Q_d adjacency, Kronecker sum of sigma_x
  signed_kron           sum of T Kronecker products of random +-1 2x2 factors,
                        symmetrised, zero diagonal (correlation-clustering weights)
  kron_sum_noise        Kronecker sum of d random symmetric U[0,1] 2x2 factors
                        plus a symmetrised Gaussian TT perturbation of rank 16
  complete, odd_cycle_plus_isolated, c5_plus_3k1: closed-form test graphs
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Graph", "grid_4x8", "kron_sum_products", "hypercube", "signed_kron",
    "kron_sum_noise", "complete", "odd_cycle_plus_isolated", "c5_plus_3k1",
    "binary_tt_adjacency", "tt_matrix_ranks",
    "config", "CONFIG_NAMES",
]


@dataclasses.dataclass
class Graph:
    """A weighted graph on n = 2^d vertices given as a TT matrix (cores) and,
    when small enough, as a dense matrix built independently of the cores."""
    name: str
    d: int
    cores: list            # list of np.float64 arrays [R, 2, 2, R']
    dense: np.ndarray | None
    meta: dict

    @property
    def n(self) -> int:
        return 2 ** self.d

    @property
    def ranks(self) -> list:
        return [c.shape[0] for c in self.cores] + [1]


# ----------------------------------------------------------------------------
# tiny core builders (graph data only)
# ----------------------------------------------------------------------------
_I2 = np.eye(2)
_SX = np.array([[0.0, 1.0], [1.0, 0.0]])


def _rank1(mats):
    """Kronecker product of 2x2 matrices as rank-1 TT cores."""
    return [np.asarray(m, dtype=np.float64).reshape(1, 2, 2, 1).copy() for m in mats]


def _tt_sum(terms, coeffs=None):
    """Block-diagonal concatenation of TT-matrix cores: the TT of sum_t c_t A_t."""
    if coeffs is None:
        coeffs = [1.0] * len(terms)
    d = len(terms[0])
    out = []
    for k in range(d):
        rl = [t[k].shape[0] for t in terms]
        rr = [t[k].shape[3] for t in terms]
        if k == 0:
            R0, R1 = 1, sum(rr)
        elif k == d - 1:
            R0, R1 = sum(rl), 1
        else:
            R0, R1 = sum(rl), sum(rr)
        G = np.zeros((R0, 2, 2, R1))
        ol = orr = 0
        for t, c in zip(terms, coeffs):
            core = t[k]
            a, b = core.shape[0], core.shape[3]
            if k == 0:
                G[0:1, :, :, orr:orr + b] = c * core if d == 1 else core
                if d == 1:
                    pass
            elif k == d - 1:
                G[ol:ol + a, :, :, 0:1] = c * core
            else:
                G[ol:ol + a, :, :, orr:orr + b] = core
            ol += a
            orr += b
        out.append(G)
    if d == 1:  # a single core: plain sum
        out = [sum(c * t[0] for t, c in zip(terms, coeffs))]
    return out


def _transpose_modes(cores):
    return [np.ascontiguousarray(c.transpose(0, 2, 1, 3)) for c in cores]


def _shift_cores(d, cyclic=False):
    """Lower shift S (S[i+1, i] = 1) as a rank-2 TT matrix.

    The bond right of core k carries the carry bit into bit k when adding one
    to the column index; core k maps (beta_k, carry_in) to alpha_k = beta_k xor
    carry_in and carry_out = beta_k and carry_in."""
    cores = []
    for k in range(d):
        G = np.zeros((2, 2, 2, 2))
        for cin in (0, 1):
            for b in (0, 1):
                a = b ^ cin
                cout = b & cin
                G[cout, a, b, cin] = 1.0
        if k == d - 1:
            G = G[:, :, :, 1:2]          # the least significant bit receives +1
        if k == 0:
            G = G.sum(axis=0, keepdims=True) if cyclic else G[0:1]
        cores.append(G)
    return cores


def _unit(d, i, j):
    """E_(i;j) as rank-1 cores (paper, Sec. 4, elementary matrices)."""
    bi = [(i >> (d - 1 - k)) & 1 for k in range(d)]
    bj = [(j >> (d - 1 - k)) & 1 for k in range(d)]
    mats = []
    for a, b in zip(bi, bj):
        m = np.zeros((2, 2))
        m[a, b] = 1.0
        mats.append(m)
    return _rank1(mats)


def _kron_dense(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def _path_dense(n):
    A = np.zeros((n, n))
    idx = np.arange(n - 1)
    A[idx + 1, idx] = 1.0
    A[idx, idx + 1] = 1.0
    return A


# ----------------------------------------------------------------------------
# graph families
# ----------------------------------------------------------------------------
def grid_4x8() -> Graph:
    """4x8 grid graph with unit weights; vertex v = 8 i + j, i in [0, 4)."""
    S2, S3 = _shift_cores(2), _shift_cores(3)
    P4 = _tt_sum([S2, _transpose_modes(S2)])
    P8 = _tt_sum([S3, _transpose_modes(S3)])
    t1 = P4 + _rank1([_I2] * 3)
    t2 = _rank1([_I2] * 2) + P8
    cores = _tt_sum([t1, t2])
    dense = np.kron(_path_dense(4), np.eye(8)) + np.kron(np.eye(4), _path_dense(8))
    return Graph("grid_4x8", 5, cores, dense, {"edges": 52})


def kron_sum_products(d=10, terms=4, seed=2) -> Graph:
    """A = K - Diag(diag K), K = sum_t kron_k F_tk, F_tk = [[a, b], [b, c]],
    a, b, c ~ U[0, 1] drawn terms-outer, modes-inner."""
    rng = np.random.default_rng(seed)
    F = np.zeros((terms, d, 2, 2))
    for t in range(terms):
        for k in range(d):
            a, b, c = rng.uniform(size=3)
            F[t, k] = [[a, b], [b, c]]
    tk = [_rank1(F[t]) for t in range(terms)]
    td = [_rank1([np.diag(np.diag(F[t, k])) for k in range(d)]) for t in range(terms)]
    cores = _tt_sum(tk + td, [1.0] * terms + [-1.0] * terms)
    dense = None
    if d <= 12:
        K = sum(_kron_dense(F[t]) for t in range(terms))
        dense = K - np.diag(np.diag(K))
    return Graph(f"kron_sum_products_d{d}_t{terms}_s{seed}", d, cores, dense,
                 {"seed": seed, "terms": terms, "factors": F})


def hypercube(d=10) -> Graph:
    """Q_d: sum over modes of I x .. x sigma_x x .. x I (Kronecker sum)."""
    terms = []
    for k in range(d):
        mats = [_I2] * d
        mats = list(mats)
        mats[k] = _SX
        terms.append(_rank1(mats))
    # compact rank-2 form of the Kronecker sum
    cores = []
    for k in range(d):
        if d == 1:
            cores.append(_SX.reshape(1, 2, 2, 1).copy())
            break
        if k == 0:
            G = np.zeros((1, 2, 2, 2)); G[0, :, :, 0] = _I2; G[0, :, :, 1] = _SX
        elif k == d - 1:
            G = np.zeros((2, 2, 2, 1)); G[0, :, :, 0] = _SX; G[1, :, :, 0] = _I2
        else:
            G = np.zeros((2, 2, 2, 2)); G[0, :, :, 0] = _I2; G[0, :, :, 1] = _SX
            G[1, :, :, 1] = _I2
        cores.append(G)
    dense = None
    if d <= 12:
        n = 2 ** d
        idx = np.arange(n)
        dense = np.zeros((n, n))
        for k in range(d):
            dense[idx, idx ^ (1 << k)] = 1.0
    return Graph(f"hypercube_d{d}", d, cores, dense, {"theta": 2.0 ** (d - 1),
                                                     "maxcut": d * 2.0 ** (d - 1)})


def signed_kron(d=12, terms=6, seed=4) -> Graph:
    """W = sym(sum_t kron_k G_tk) with zero diagonal, G_tk entries in {-1, +1}
    drawn as integers(0, 2, (2, 2)) * 2 - 1, terms-outer, modes-inner."""
    rng = np.random.default_rng(seed)
    G = np.zeros((terms, d, 2, 2))
    for t in range(terms):
        for k in range(d):
            G[t, k] = rng.integers(0, 2, (2, 2)) * 2 - 1
    t0 = [_rank1(G[t]) for t in range(terms)]
    t0T = [_transpose_modes(c) for c in t0]
    td = [_rank1([np.diag(np.diag(G[t, k])) for k in range(d)]) for t in range(terms)]
    cores = _tt_sum(t0 + t0T + td, [0.5] * terms + [0.5] * terms + [-1.0] * terms)
    dense = None
    if d <= 12:
        W0 = sum(_kron_dense(G[t]) for t in range(terms))
        W = 0.5 * (W0 + W0.T)
        dense = W - np.diag(np.diag(W))
    return Graph(f"signed_kron_d{d}_t{terms}_s{seed}", d, cores, dense,
                 {"seed": seed, "terms": terms, "factors": G})


def _tt_fro2(cores):
    """Squared Frobenius norm of a TT matrix by contracting the network."""
    E = np.ones((1, 1))
    for G in cores:
        E = np.einsum("ab,aijc,bijd->cd", E, G, G)
    return float(E[0, 0])


def kron_sum_noise(d=12, seed=5, noise_rank=16, sigma=0.1) -> Graph:
    """A = (Kronecker sum of F_k) + P_s, F_k = [[a, b], [b, c]] ~ U[0, 1];
    P a TT matrix with interior ranks noise_rank and N(0, 1) core entries,
    P_s = (P + P^T)/2 scaled so that ||P_s||_F / n = sigma.  Draw order: the
    three uniforms of each F_k in mode order, then the cores of P in mode order."""
    rng = np.random.default_rng(seed)
    F = np.zeros((d, 2, 2))
    for k in range(d):
        a, b, c = rng.uniform(size=3)
        F[k] = [[a, b], [b, c]]
    P = []
    for k in range(d):
        rl = 1 if k == 0 else noise_rank
        rr = 1 if k == d - 1 else noise_rank
        P.append(rng.standard_normal((rl, 2, 2, rr)))
    Ps = _tt_sum([P, _transpose_modes(P)], [0.5, 0.5])
    n = 2 ** d
    scale = sigma * n / np.sqrt(_tt_fro2(Ps))
    Ps[-1] = Ps[-1] * scale
    ks = []
    for k in range(d):
        mats = [_I2] * d
        mats = list(mats)
        mats[k] = F[k]
        ks.append(_rank1(mats))
    cores = _tt_sum(ks + [Ps])
    dense = None
    if d <= 12:
        K = sum(_kron_dense([F[j] if j == k else _I2 for j in range(d)]) for k in range(d))
        # dense P from its cores (plain reshape-contract, big-endian)
        M = np.ones((1, 1, 1))
        for G in P:
            M = np.einsum("abr,rijs->aibjs", M, G).reshape(M.shape[0] * 2, M.shape[1] * 2, G.shape[3])
        Pd = M[:, :, 0]
        dense = K + scale * 0.5 * (Pd + Pd.T)
    return Graph(f"kron_sum_noise_d{d}_s{seed}", d, cores, dense,
                 {"seed": seed, "factors": F, "noise_rank": noise_rank, "sigma": sigma,
                  "scale": scale})


def complete(d) -> Graph:
    """K_n, n = 2^d: J - I (MaxCut value n^2/4)."""
    J = _rank1([np.ones((2, 2))] * d)
    I = _rank1([_I2] * d)
    cores = _tt_sum([J, I], [1.0, -1.0])
    n = 2 ** d
    return Graph(f"complete_d{d}", d, cores, np.ones((n, n)) - np.eye(n),
                 {"maxcut": n * n / 4.0})


def odd_cycle_plus_isolated(d) -> Graph:
    """Cycle on the first n-1 = 2^d - 1 vertices plus one isolated vertex.
    MaxCut SDP value (m/2)(1 + cos(pi/m)) with m = n - 1."""
    n = 2 ** d
    S = _shift_cores(d)
    path = [S, _transpose_modes(S)]
    extra = [_unit(d, n - 1, n - 2), _unit(d, n - 2, n - 1), _unit(d, 0, n - 2), _unit(d, n - 2, 0)]
    cores = _tt_sum(path + extra, [1.0, 1.0, -1.0, -1.0, 1.0, 1.0])
    m = n - 1
    dense = np.zeros((n, n))
    for v in range(m):
        w = (v + 1) % m
        dense[v, w] = dense[w, v] = 1.0
    return Graph(f"odd_cycle_{m}_plus_k1", d, cores, dense,
                 {"maxcut": m / 2.0 * (1.0 + np.cos(np.pi / m))})


def c5_plus_3k1() -> Graph:
    """C_5 on vertices 0..4 plus three isolated vertices (n = 8); theta = 3 + sqrt 5."""
    d, n = 3, 8
    edges = [(v, (v + 1) % 5) for v in range(5)]
    terms = []
    for u, v in edges:
        terms += [_unit(d, u, v), _unit(d, v, u)]
    cores = _tt_sum(terms)
    dense = np.zeros((n, n))
    for u, v in edges:
        dense[u, v] = dense[v, u] = 1.0
    return Graph("c5_plus_3k1", d, cores, dense, {"theta": 3.0 + np.sqrt(5.0)})


def tt_matrix_ranks(cores, rtol=1e-10):
    """TT ranks of a TT matrix after compression (right-to-left QR, then
    left-to-right SVD keeping singular values above rtol times the largest)."""
    G = [np.asarray(c, dtype=np.float64) for c in cores]
    d = len(G)
    for k in range(d - 1, 0, -1):
        R0, m1, m2, R1 = G[k].shape
        Q, Rt = np.linalg.qr(G[k].reshape(R0, -1).T)
        G[k] = Q.T.reshape(-1, m1, m2, R1)
        G[k - 1] = np.tensordot(G[k - 1], Rt.T, axes=(3, 0))
    ranks = [1]
    for k in range(d - 1):
        R0, m1, m2, R1 = G[k].shape
        U, sv, Vt = np.linalg.svd(G[k].reshape(R0 * m1 * m2, R1), full_matrices=False)
        keep = max(1, int(np.sum(sv > rtol * sv[0]))) if sv.size and sv[0] > 0 else 1
        G[k] = U[:, :keep].reshape(R0, m1, m2, keep)
        G[k + 1] = np.tensordot(sv[:keep, None] * Vt[:keep], G[k + 1], axes=(1, 0))
        ranks.append(keep)
    return ranks + [1]


def binary_tt_adjacency(d, r, seed=0, bias=0.0, max_tries=500) -> Graph:
    """Random simple graph (symmetric 0/1 adjacency, zero diagonal) of TT rank r
    on 2^d vertices, by the construction of the paper's App. A ("Sampling
    Binary TT Matrices", "Sampling Adjacency TT Matrices without
    Self-Connections").

    An orthonormal basis q_0..q_{r-1} (rows of Q, QR of a Gaussian matrix)
    carries a path state through the cores.  The first core puts basis row
    q_i(alpha, beta) on mode pair (alpha, beta); each middle core applies, per
    mode pair, P = I + sum_i q_i (q_sigma(i) - q_i)^T, which sends q_i to
    q_sigma(i) (sigma a random map of the basis indices); the last core reads
    the state against q_j(alpha, beta), giving 1 for the same basis vector and
    0 for an orthogonal one.  Entries are therefore 0/1 and the TT rank is at
    most r.  Symmetry: the (alpha, beta) and (beta, alpha) slices of every
    core are equal.  Zero diagonal: the diagonal slice of the second core
    drops the states that all-diagonal prefixes can reach (the term
    - sum_{i in D} q_i q_i^T of the paper), so every diagonal entry is 0 (for
    d = 2 the last core avoids those states instead).  The indices i, sigma(i),
    j are drawn with weights exp(-bias * index) (bias = 0: uniform; a larger
    bias gives fewer orthogonal combinations and denser graphs).  Samples are
    rejected until the TT rank is exactly r and the graph has an edge.

    Reading: the paper does not state the pair distribution, the number of
    pairs or the rejection details; sigma is a full random map here, so
    instances match the paper's in distribution type, not sample by sample."""
    if d < 2 or r < 1:
        raise ValueError("need d >= 2 and r >= 1")
    rng = np.random.default_rng(seed)
    pairs = [(0, 0), (0, 1), (1, 1)]
    for _ in range(max_tries):
        Q, _ = np.linalg.qr(rng.standard_normal((r, r)))
        w = np.exp(-bias * np.arange(r))
        w /= w.sum()
        first = {}
        for a, b in pairs:
            first[(a, b)] = first[(b, a)] = int(rng.choice(r, p=w))
        diag_states = {first[(0, 0)], first[(1, 1)]}
        maps = []
        for _k in range(1, d - 1):
            m = {}
            for a, b in pairs:
                sigma = rng.choice(r, size=r, p=w).astype(np.int64)
                if a == b:
                    for i in diag_states:
                        sigma[i] = -1          # cancelled: all-diagonal prefixes end here
                m[(a, b)] = m[(b, a)] = sigma
            maps.append(m)
            diag_states = set()
        last = {}
        for a, b in pairs:
            choices = [j for j in range(r) if a != b or j not in diag_states]
            if not choices:
                last[(a, b)] = last[(b, a)] = -1
                continue
            ww = w[choices] / w[choices].sum()
            last[(a, b)] = last[(b, a)] = int(choices[int(rng.choice(len(choices), p=ww))])
        # TT cores
        cores = []
        G = np.zeros((1, 2, 2, r))
        for (a, b), i in first.items():
            G[0, a, b, :] = Q[i]
        cores.append(G)
        for m in maps:
            G = np.zeros((r, 2, 2, r))
            for (a, b), sigma in m.items():
                for i in range(r):
                    if sigma[i] >= 0:
                        G[:, a, b, :] += np.outer(Q[i], Q[sigma[i]])
            cores.append(G)
        G = np.zeros((r, 2, 2, 1))
        for (a, b), j in last.items():
            if j >= 0:
                G[:, a, b, 0] = Q[j]
        cores.append(G)
        # dense adjacency by following the path states (independent of the TT contraction)
        dense = None
        if d <= 12:
            n = 2 ** d
            u = np.arange(n)[:, None] + np.zeros((1, n), dtype=np.int64)
            v = np.arange(n)[None, :] + np.zeros((n, 1), dtype=np.int64)
            bit = lambda x, k: (x >> (d - 1 - k)) & 1
            ua, vb = bit(u, 0), bit(v, 0)
            state = np.zeros((n, n), dtype=np.int64)
            for (a, b), i in first.items():
                state[(ua == a) & (vb == b)] = i
            for k, m in enumerate(maps, start=1):
                ua, vb = bit(u, k), bit(v, k)
                new = np.full((n, n), -1, dtype=np.int64)
                for (a, b), sigma in m.items():
                    sel = (ua == a) & (vb == b) & (state >= 0)
                    new[sel] = sigma[state[sel]]
                state = new
            ua, vb = bit(u, d - 1), bit(v, d - 1)
            dense = np.zeros((n, n))
            for (a, b), j in last.items():
                sel = (ua == a) & (vb == b) & (state >= 0) & (state == j)
                dense[sel] = 1.0
            if dense.sum() == 0:
                continue
        if max(tt_matrix_ranks(cores)) != r:
            continue
        return Graph(f"binary_tt_d{d}_r{r}_s{seed}", d, cores, dense,
                     {"seed": seed, "tt_rank": r, "bias": bias})
    raise RuntimeError(f"no graph of TT rank {r} on 2^{d} vertices after {max_tries} draws")


# ----------------------------------------------------------------------------
# the five benchmark configurations (problem kind, graph, rank cap, precision)
# ----------------------------------------------------------------------------
CONFIG_NAMES = ["maxcut_grid_d5", "maxcut_kron_d10", "theta_hypercube_d10",
                "cc_signed_d12", "maxcut_noise_d12"]


def negdeg_cores(g: Graph, tol=1e-14):
    """TT cores (mode 2) of the negative-degree vector C^- 1 of a signed graph,
    C^- = max(-W, 0), by successive truncated SVDs at relative tol (the input
    of the correlation-clustering encoding)."""
    v = np.maximum(-g.dense, 0.0).sum(axis=1)
    cores, r, C = [], 1, np.asarray(v, dtype=np.float64).reshape(1, -1)
    for k in range(g.d - 1):
        C = C.reshape(r * 2, -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = max(1, int(np.sum(s > tol * max(s[0], 1e-300))))
        cores.append(U[:, :rk].reshape(r, 2, rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, 2, 1))
    return cores


def config(name: str) -> dict:
    if name == "maxcut_grid_d5":
        return {"kind": "maxcut", "graph": grid_4x8(), "rank_cap": 8, "precision": "f64"}
    if name == "maxcut_kron_d10":
        return {"kind": "maxcut", "graph": kron_sum_products(10, 4, 2), "rank_cap": 32,
                "precision": "f64"}
    if name == "theta_hypercube_d10":
        return {"kind": "theta", "graph": hypercube(10), "rank_cap": 64, "precision": "mixed"}
    if name == "cc_signed_d12":
        return {"kind": "cc", "graph": signed_kron(12, 6, 4), "rank_cap": 64,
                "precision": "mixed"}
    if name == "maxcut_noise_d12":
        return {"kind": "maxcut", "graph": kron_sum_noise(12, 5), "rank_cap": 128,
                "precision": "mixed"}
    raise KeyError(name)
