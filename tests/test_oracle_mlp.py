"""Pins of the MLP oracle: finite differences, the BCE-gradient closed form, lstsq."""
import numpy as np

from oracle import mlp
from tests.conftest import planted, rand_dicts


def small_net(rng, M=8, H=6, A=5):
    _, n = mlp.layout(M, H, A)
    return rng.standard_normal(n) * 0.5, M, H, A


def test_gradient_matches_central_differences(rng):
    p, M, H, A = small_net(rng)
    x = rng.standard_normal((7, M))
    y = (rng.random((7, A)) < 0.3).astype(float)
    _, g = mlp.loss_and_grad(p, x, y, M, H, A)
    h = 1e-6
    for i in rng.choice(p.size, 40, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, x, y, M, H, A)
        lm, _ = mlp.loss_and_grad(p - e, x, y, M, H, A)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))


def test_logit_gradient_closed_form(rng):
    # d(mean BCE)/dz = (sigmoid(z) - y) / (B*A); check through the output bias gradient
    p, M, H, A = small_net(rng)
    x = rng.standard_normal((4, M))
    y = (rng.random((4, A)) < 0.5).astype(float)
    z, _ = mlp.forward(p, x, M, H, A)
    _, g = mlp.loss_and_grad(p, x, y, M, H, A)
    off, _ = mlp.layout(M, H, A)
    np.testing.assert_allclose(g[off[5]:off[6]], ((1 / (1 + np.exp(-z)) - y) / (4 * A)).sum(0), rtol=1e-12)


def test_gelu_is_z_times_normal_cdf():
    from scipy.stats import norm
    z = np.linspace(-5, 5, 101)
    np.testing.assert_allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-12, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-8)


def test_top_s_ties_and_ls(rng):
    z = np.array([[1.0, 3.0, 3.0, 0.5, 3.0]])
    np.testing.assert_array_equal(mlp.top_s(z, 3), [[1, 2, 4]])
    d1, d2 = rand_dicts(rng, 4, 4, 5, 5)
    Y, _ = planted(rng, 6, d1, d2, 3, noise=0.0)
    supp = np.array([rng.choice(25, 3, replace=False) for _ in range(6)])
    coef, res2 = mlp.least_squares_on_support(Y, d1, d2, supp)
    K = np.kron(d2, d1)
    for k in range(6):
        r = Y[k].flatten("F") - K[:, supp[k]] @ coef[k]
        np.testing.assert_allclose(K[:, supp[k]].T @ r, 0, atol=1e-12)
        np.testing.assert_allclose(res2[k], r @ r, rtol=1e-12, atol=1e-20)


def test_inputs_are_unit_norm_colmajor(rng):
    Y = rng.standard_normal((3, 4, 5))
    x = mlp.inputs(Y)
    np.testing.assert_allclose(np.linalg.norm(x, axis=1), 1.0)
    np.testing.assert_allclose(x[0], Y[0].flatten("F") / np.linalg.norm(Y[0]))
