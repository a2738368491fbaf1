"""Pins of the oracle's Karhunen-Loeve expansion (separable exponential
covariance on the unit square; the truncated KL expansion of Sec. 5).

The eigenpairs are checked against what the integral operator itself fixes:
a Nystrom discretisation, orthonormality, the eigen-equation residual, the
Robin boundary conditions of the equivalent ODE, and the operator trace.
"""
import numpy as np
import pytest

import oracle

CORRS = [0.3, 0.1]


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


def _nystrom(corr, n, k):
    t = (np.arange(n) + 0.5) / n
    Cm = np.exp(-np.abs(t[:, None] - t[None, :]) / corr) / n
    return np.sort(np.linalg.eigvalsh(Cm))[::-1][:k]


@pytest.mark.parametrize("corr", CORRS)
def test_eigenvalues_match_nystrom(corr):
    _, mu = oracle.kl_roots_1d(8, corr)
    e1 = _nystrom(corr, 1200, 8)
    e2 = _nystrom(corr, 2400, 8)
    rich = (4 * e2 - e1) / 3  # midpoint rule error is O(n^-2)
    np.testing.assert_allclose(mu, rich, rtol=2e-7)


@pytest.mark.parametrize("corr", CORRS)
def test_eigenfunctions_orthonormal(corr):
    om, _ = oracle.kl_roots_1d(12, corr)
    t, w = _gl(400, 0.0, 1.0)
    Phi = np.array([oracle.kl_phi_1d(o, corr, t) for o in om])
    G = (Phi * w) @ Phi.T
    np.testing.assert_allclose(G, np.eye(12), atol=1e-12)


@pytest.mark.parametrize("corr", CORRS)
def test_eigen_equation_residual(corr):
    om, mu = oracle.kl_roots_1d(10, corr)
    for o, m in zip(om, mu):
        for s in [0.0, 0.137, 0.5, 0.8, 1.0]:
            acc = 0.0
            for a, b in [(0.0, s), (s, 1.0)]:
                if b > a:
                    t, w = _gl(200, a, b)
                    acc += np.sum(w * np.exp(-np.abs(s - t) / corr) * oracle.kl_phi_1d(o, corr, t))
            assert abs(acc - m * oracle.kl_phi_1d(o, corr, [s])[0]) < 1e-11


@pytest.mark.parametrize("corr", CORRS)
def test_robin_boundary_conditions_and_sign(corr):
    om, _ = oracle.kl_roots_1d(6, corr)
    c = 1.0 / corr
    h = 1e-3
    for o in om:
        f = lambda t: oracle.kl_phi_1d(o, corr, [t])[0]
        d0 = (f(-2 * h) - 8 * f(-h) + 8 * f(h) - f(2 * h)) / (12 * h)
        d1 = (f(1 - 2 * h) - 8 * f(1 - h) + 8 * f(1 + h) - f(1 + 2 * h)) / (12 * h)
        assert abs(d0 - c * f(0.0)) < 1e-7 * max(1, o)
        assert abs(d1 + c * f(1.0)) < 1e-7 * max(1, o)
        assert f(0.0) > 0


def test_roots_bracketed_and_trace():
    corr = 0.3
    N = 3000
    om, mu = oracle.kl_roots_1d(N, corr)
    n = np.arange(1, N + 1)
    assert np.all((om > (n - 1) * np.pi) & (om < n * np.pi))
    # trace of the operator on [0,1] is 1; the tail beyond N modes is about
    # sum_{n>N} 2c/(n pi)^2 ~ 2c/(pi^2 N)
    tail = 1.0 - mu.sum()
    est = 2 / corr / (np.pi ** 2 * N)
    assert 0 < tail < 1.5 * est and tail > 0.5 * est


def test_2d_modes_order_and_products():
    K, s2, corr = 60, 1.7, 0.3
    lam, ix, iy, ox, oy = oracle.kl_modes_2d(K, s2, corr)
    om, mu = oracle.kl_roots_1d(K, corr)
    assert np.all(np.diff(lam) <= 0)
    np.testing.assert_array_equal(lam, s2 * (mu[ix] * mu[iy]))
    np.testing.assert_array_equal(ox, om[ix])
    # the K largest products of all pairs, as a multiset
    allp = np.sort((s2 * (mu[:, None] * mu[None, :])).ravel())[::-1][:K]
    np.testing.assert_array_equal(np.sort(lam)[::-1], allp)
    # exact ties (i,j)/(j,i): smaller i first
    ties = 0
    for k in range(K - 1):
        if lam[k] == lam[k + 1]:
            assert ix[k] < ix[k + 1]
            ties += 1
    assert ties >= K // 3  # the (i,j)/(j,i) pairs tie exactly
    assert ix[0] == 0 and iy[0] == 0


def _centroid_from_vertices(l):
    n = 1 << l
    out = []
    for j in range(n):
        for i in range(n):
            lo = [(i, j), (i + 1, j), (i + 1, j + 1)]
            up = [(i, j), (i + 1, j + 1), (i, j + 1)]
            for tri in (lo, up):
                out.append((sum(v[0] for v in tri) / (3 * n), sum(v[1] for v in tri) / (3 * n)))
    return np.array(out)


@pytest.mark.parametrize("l", [1, 2, 3, 5])
def test_centroids(l):
    np.testing.assert_allclose(oracle.centroids(l), _centroid_from_vertices(l), rtol=0, atol=1e-15)


def test_basis_is_separable_product():
    l, K, s2, corr = 3, 12, 1.0, 0.3
    B = oracle.kl_basis(l, K, s2, corr)
    lam, ix, iy, ox, oy = oracle.kl_modes_2d(K, s2, corr)
    xy = oracle.centroids(l)
    for k in range(K):
        ref = np.sqrt(lam[k]) * oracle.kl_phi_1d(ox[k], corr, xy[:, 0]) * oracle.kl_phi_1d(oy[k], corr, xy[:, 1])
        np.testing.assert_allclose(B[k], ref, rtol=1e-14, atol=1e-15)


def test_field_is_matrix_product():
    from tests import inputs
    l, K = 3, 10
    B = oracle.kl_basis(l, K, 1.0, 0.3)
    th = inputs.theta_batch(3, 7, K)
    np.testing.assert_allclose(oracle.kl_field(l, B, th), th @ B, rtol=1e-13, atol=1e-14)


def test_truncated_field_variance():
    # pointwise variance of the truncated field sum_k lambda_k phi_k(x)^2
    # approaches sigma2 from below as K grows (Mercer)
    l, corr = 3, 0.3
    v_prev = None
    for K in [10, 50, 200]:
        B = oracle.kl_basis(l, K, 1.0, corr)
        v = (B ** 2).sum(0)
        assert np.all(v < 1.0 + 1e-12)
        if v_prev is not None:
            assert np.all(v >= v_prev - 1e-15)
        v_prev = v
    assert v_prev.mean() > 0.9
