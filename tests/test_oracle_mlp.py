"""Pins of the MLP reference (learned block preconditioner): hand-derived
gradients against central finite differences, and a closed-form optimum."""
import numpy as np

from oracle import mlp


def _data(rng, N=5, P=3, n=4, in_dim=7):
    F = rng.standard_normal((N, in_dim))
    R = rng.standard_normal((N, P, n))
    Y = rng.standard_normal((N, P, n))
    S = rng.uniform(0.5, 2.0, N)
    Wt = rng.uniform(0.5, 1.5, (N, P))
    return F, R, Y, S, Wt


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    n, in_dim, H = 4, 7, 9
    F, R, Y, S, Wt = _data(rng, n=n, in_dim=in_dim)
    params = mlp.init_params(in_dim, H, n * n, seed=1, out_scale=1.0)
    # move the biases off zero so that every ReLU is differentiable at the point
    params["b1"] += 0.1
    params["b2"] += 0.1
    _, g = mlp.loss_and_grad(params, F, R, Y, S, Wt)
    for name in mlp.PARAM_ORDER:
        flat = params[name].reshape(-1)
        for k in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            idx = np.unravel_index(k, params[name].shape)
            fd = mlp.finite_difference(params, F, R, Y, S, Wt, name, idx)
            assert abs(fd - g[name][idx]) <= 1e-6 * (1 + abs(fd)), (name, idx, fd, g[name][idx])


def test_zero_loss_and_gradient_at_exact_correction():
    """If every block's BJ residual is exactly (1/s) C* y for one matrix C*, the
    network with W3 = 0, b3 = vec(C*) has zero loss and zero gradient."""
    rng = np.random.default_rng(3)
    n, in_dim, H, N, P = 3, 5, 6, 4, 4
    Cstar = rng.standard_normal((n, n))
    F = rng.standard_normal((N, in_dim))
    Y = rng.standard_normal((N, P, n))
    S = rng.uniform(0.5, 2.0, N)
    R = np.einsum("ij,bpj->bpi", Cstar, Y) / S[:, None, None]
    Wt = np.ones((N, P))
    params = mlp.init_params(in_dim, H, n * n, seed=2)
    params["b3"] = Cstar.reshape(-1).copy()
    loss, g = mlp.loss_and_grad(params, F, R, Y, S, Wt)
    assert loss < 1e-28
    for name in mlp.PARAM_ORDER:
        assert np.abs(g[name]).max() < 1e-13


def test_flatten_roundtrip():
    params = mlp.init_params(6, 8, 9, seed=4, out_scale=0.5)
    back = mlp.unflatten(mlp.flatten(params), 6, 8, 9)
    for k in mlp.PARAM_ORDER:
        assert np.array_equal(back[k], params[k])
