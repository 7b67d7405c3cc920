"""Reference (FP64, NumPy) of the learned block preconditioner's network.

Test infrastructure only: the GPU library never imports this module.

The network maps the features f of one diagonal block (a, b) of a local
system (the normalised block entries and a few scalars) to a correction C of
the block-Jacobi inverse: the preconditioner block is B^{-1} + C / s with s the
block's Frobenius norm.  Two hidden layers with ReLU:
    z1 = W1 f + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2), out = W3 h2 + b3,
C = out reshaped n x n (row-major).

Loss of a batch of N blocks, each with P probe pairs (r_i, y_i) and weights
w_i: with y = K x for a probe x of the whole local system, y_b its block and
r_b = x_b - B^{-1} y_b the block-Jacobi residual,
    L = (1/N) sum_blocks sum_i w_i || r_i - (1/s) C y_i ||^2,
i.e. the block part of || x - M K x ||^2 for the left-preconditioned
operator M K: a block-diagonal M that makes M K close to the identity on the
probes.  Gradients are derived by hand (backpropagation written out below);
a central finite-difference check pins them.
"""
import numpy as np


def init_params(in_dim, hidden, out_dim, seed=0, out_scale=0.0):
    """He-initialised hidden layers; the output layer starts at out_scale * N(0, 1/H)
    (0 gives the plain block-Jacobi preconditioner at initialisation)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((hidden, in_dim)) * np.sqrt(2.0 / in_dim),
        "b1": np.zeros(hidden),
        "W2": rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden),
        "b2": np.zeros(hidden),
        "W3": rng.standard_normal((out_dim, hidden)) * (out_scale / np.sqrt(hidden)),
        "b3": np.zeros(out_dim),
    }


def forward(params, F):
    """F: (N, in_dim) -> (out (N, out_dim), cache)."""
    z1 = F @ params["W1"].T + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["W2"].T + params["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ params["W3"].T + params["b3"]
    return out, (F, z1, h1, z2, h2)


def loss_and_grad(params, F, R, Y, S, Wt):
    """F (N, in), R and Y (N, P, n), S (N,), Wt (N, P).  Returns (loss, grads)."""
    N, P, n = R.shape
    out, (F_, z1, h1, z2, h2) = forward(params, F)
    C = out.reshape(N, n, n)
    CY = np.einsum("bij,bpj->bpi", C, Y) / S[:, None, None]
    E = R - CY                                             # (N, P, n)
    loss = float(np.sum(Wt[:, :, None] * E * E) / N)
    # dL/dC_b = -(2/N)(1/s_b) sum_p w_p e_p y_p^T
    dC = -(2.0 / N) * np.einsum("bp,bpi,bpj->bij", Wt, E, Y) / S[:, None, None]
    dout = dC.reshape(N, n * n)
    g = {}
    g["W3"] = dout.T @ h2
    g["b3"] = dout.sum(0)
    dh2 = dout @ params["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ params["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ F_
    g["b1"] = dz1.sum(0)
    return loss, g


def finite_difference(params, F, R, Y, S, Wt, name, idx, h=1e-6):
    """Central difference of the loss in one parameter entry."""
    p_plus = {k: v.copy() for k, v in params.items()}
    p_minus = {k: v.copy() for k, v in params.items()}
    p_plus[name][idx] += h
    p_minus[name][idx] -= h
    lp, _ = loss_and_grad(p_plus, F, R, Y, S, Wt)
    lm, _ = loss_and_grad(p_minus, F, R, Y, S, Wt)
    return (lp - lm) / (2 * h)


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(params):
    return np.concatenate([params[k].reshape(-1) for k in PARAM_ORDER])


def unflatten(vec, in_dim, hidden, out_dim):
    shapes = {"W1": (hidden, in_dim), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (out_dim, hidden), "b3": (out_dim,)}
    out, off = {}, 0
    for k in PARAM_ORDER:
        sz = int(np.prod(shapes[k]))
        out[k] = np.asarray(vec[off:off + sz], dtype=np.float64).reshape(shapes[k])
        off += sz
    return out
