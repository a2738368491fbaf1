"""Pins of the oracle MLP (the surrogate's reference): gradients against
central finite differences of the oracle's own loss, GELU against its
defining integral, and the forward pass against a layer-by-layer numpy
evaluation with scipy's erf."""
import numpy as np
from scipy.special import erf

import oracle
from tests import inputs


def _params(dims, seed):
    D, H1, H2, O = dims
    n = H1 * D + H1 + H2 * H1 + H2 + O * H2 + O
    return 0.3 * inputs.rng(seed).standard_normal(n)


def test_forward_matches_numpy_layers():
    dims = (6, 9, 7, 4)
    D, H1, H2, O = dims
    P = _params(dims, 0)
    x = inputs.rng(1).standard_normal((5, D))
    W1 = P[:H1 * D].reshape(H1, D); o = H1 * D
    b1 = P[o:o + H1]; o += H1
    W2 = P[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = P[o:o + H2]; o += H2
    W3 = P[o:o + O * H2].reshape(O, H2); o += O * H2
    b3 = P[o:o + O]
    g = lambda z: 0.5 * z * (1 + erf(z / np.sqrt(2)))
    ref = g(g(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    np.testing.assert_allclose(oracle.mlp_forward(dims, P, x), ref, rtol=1e-13, atol=1e-14)


def test_gelu_is_z_times_normal_cdf():
    # GELU(z) = z * P(Z <= z): check the CDF by quadrature of the density
    from scipy.integrate import quad
    dims = (1, 1, 1, 1)
    for z in [-2.0, -0.3, 0.0, 0.7, 2.5]:
        cdf = quad(lambda t: np.exp(-t * t / 2) / np.sqrt(2 * np.pi), -np.inf, z)[0]
        # a network that is the identity around one GELU: W1 = 1, b1 = 0,
        # W2 = 1, b2 = big so the second GELU is ~linear, W3 = 1, b3 = -big
        big = 40.0
        P = np.array([1.0, 0.0, 1.0, big, 1.0, -big])
        out = oracle.mlp_forward(dims, P, np.array([[z]]))[0, 0]
        assert abs(out - z * cdf) < 1e-12


def test_gradient_central_differences():
    dims = (5, 8, 6, 3)
    P = _params(dims, 2)
    x = inputs.rng(3).standard_normal((4, dims[0]))
    t = inputs.rng(4).standard_normal((4, dims[3]))
    loss, g = oracle.mlp_loss_grad(dims, P, x, t)
    assert abs(loss - 0.5 * np.mean((oracle.mlp_forward(dims, P, x) - t) ** 2)) < 1e-14
    h = 1e-6
    fd = np.zeros_like(P)
    for i in range(len(P)):
        Pp = P.copy(); Pp[i] += h
        Pm = P.copy(); Pm[i] -= h
        fd[i] = (oracle.mlp_loss_grad(dims, Pp, x, t)[0] - oracle.mlp_loss_grad(dims, Pm, x, t)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
