"""Pins of the FP64 surrogate-network reference: backpropagation against central
finite differences, and the GELU derivative against its difference quotient."""
import numpy as np

from oracle import mlp_ref


def test_gelu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp_ref.gelu(z + h) - mlp_ref.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp_ref.gelu_prime(z), fd, rtol=1e-7, atol=1e-8)
    # GELU(z) -> z for large z, -> 0 for very negative z
    assert abs(mlp_ref.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    assert abs(mlp_ref.gelu(np.array([-8.0]))[0]) < 1e-12


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = rng.normal(0, 0.2, mlp_ref.NPARAM)
    X = rng.uniform(-1, 1, (16, 6))
    t = rng.normal(0, 1, 16)
    loss, g = mlp_ref.loss_and_grad(theta, X, t)
    assert g.size == mlp_ref.NPARAM == 34049
    idx = rng.choice(mlp_ref.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp_ref.NPARAM - 1, 0, 800, 20000]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp_ref.loss_and_grad(theta + e, X, t)[0] - mlp_ref.loss_and_grad(theta - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
