"""Pins of the oracle's Matern (nu = 3/2) KL expansion by the Nystrom method
(the prior of Sec. 5, Examples 5.1-5.3).

What fixes it besides its own formulas: the Bessel-function form of the
Matern covariance, the spectrum of the whole Nystrom matrix (the parity
classes must reproduce it), the eigen equation, the operator trace, the
midpoint rule's convergence, and the variance fractions the paper prints.
The fractions also fix the length-scale convention: the argument r/lam
gives 0.957 and 0.995 for the first two rows of the golden file, sqrt(3)
r/lam gives 0.869 and 0.977; only 2 sqrt(nu) r/lam = sqrt(6) r/lam holds
0.764 and 0.945.
"""
import os

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import matern

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "matern_kl_variance_fractions.txt")


def _golden():
    rows = []
    for ln in open(GOLDEN):
        if ln.startswith("#") or not ln.strip():
            continue
        f = ln.split()
        rows.append((float(f[0]), int(f[1]), float(f[2]), float(f[3]), " ".join(f[4:])))
    return rows


def test_kernel_is_the_bessel_form():
    nu, lam, s2 = 1.5, 0.37, 1.7
    r = np.linspace(1e-3, 2.0, 97)
    z = 2.0 * np.sqrt(nu) * r / lam
    ref = s2 * 2.0 ** (1 - nu) / special.gamma(nu) * z ** nu * special.kv(nu, z)
    np.testing.assert_allclose(matern.matern32(r, lam, s2), ref, rtol=1e-13)
    assert matern.matern32(0.0, lam, s2) == s2


@pytest.mark.parametrize("m,lam", [(12, 0.3), (16, 0.65), (16, 0.1)])
def test_parity_classes_reproduce_the_full_spectrum(m, lam):
    A = matern.full_matrix(m, lam, 1.3)
    full = np.sort(np.linalg.eigvalsh(A))[::-1]
    lam_k, V, cls = matern.modes(m * m, m, lam, 1.3)
    np.testing.assert_allclose(lam_k, full, rtol=1e-11, atol=1e-15 * full[0])
    R = A @ V - V * lam_k
    assert np.abs(R).max() < 1e-13 * full[0]
    np.testing.assert_allclose(V.T @ V, np.eye(m * m), atol=1e-12)


def test_canonical_basis_rules():
    m, lam = 16, 0.3
    lam_k, V, cls = matern.modes(40, m, lam)
    q1 = np.arange(m * m) + 1.0
    g = np.modf(q1 * q1 * matern.GOLDEN_FRAC)[0] - 0.5
    assert np.all(g @ V > 0)
    grid = V.reshape(m, m, -1)  # [b, a, k]
    for k in range(40):
        sx, sy = matern.CLASSES[cls[k]]
        np.testing.assert_allclose(grid[:, ::-1, k], sx * grid[:, :, k], atol=1e-14)
        np.testing.assert_allclose(grid[::-1, :, k], sy * grid[:, :, k], atol=1e-14)
    assert np.all(np.diff(lam_k) <= 0)
    # the swapped classes pair up with exactly equal eigenvalues, (-,+) first
    for k in np.nonzero(cls == 1)[0]:
        j = np.nonzero((cls == 2) & (lam_k == lam_k[k]))[0]
        if k + 1 < 40:
            assert j.size == 1 and j[0] == k + 1


@pytest.mark.parametrize("m", [4, 6, 8, 12, 16, 24, 32])
def test_sign_rule_is_well_conditioned(m):
    """|g.v| must stay far above rounding for every mode, or the sign (and
    so the basis) would depend on the order of floating-point operations.
    The quadratic sequence keeps it above 2e-4 here; a linear one vanishes
    for the modes odd under the diagonal swap on small grids."""
    _, V, _ = matern.modes(min(m * m, 200), m, 0.3)
    q1 = np.arange(m * m) + 1.0
    g = np.modf(q1 * q1 * matern.GOLDEN_FRAC)[0] - 0.5
    assert np.abs(g @ V).min() > 1e-4
    g_lin = np.modf(q1 * matern.GOLDEN_FRAC)[0] - 0.5
    if m in (4, 6):
        assert np.abs(g_lin @ V).min() < 1e-12


def test_trace_is_the_variance():
    lam_k, _, _ = matern.modes(256, 16, 0.2, 2.5)
    assert abs(lam_k.sum() - 2.5) < 1e-12


@pytest.mark.parametrize("lam,K,printed,tol,where", _golden())
def test_paper_variance_fractions(lam, K, printed, tol, where):
    m = 48 if lam > 0.3 else 64
    lam_k, _, _ = matern.modes(K, m, lam)
    assert abs(lam_k.sum() - printed) <= tol, (lam_k.sum(), where)


def test_midpoint_rule_converges():
    a, _, _ = matern.modes(12, 24, 0.65)
    b, _, _ = matern.modes(12, 48, 0.65)
    c, _, _ = matern.modes(12, 96, 0.65)
    # O(h^2): the error shrinks about fourfold per halving of h
    e1, e2 = np.abs(a - c), np.abs(b - c)
    assert np.all(e2 < 0.4 * e1 + 1e-12)
    assert np.all(np.abs(b - c) < 2e-3 * c)


def test_extension_interpolates_the_nodes():
    m, lam = 16, 0.3
    lam_k, V, _ = matern.modes(20, m, lam)
    P = matern.points(m)
    B = matern.extend(P, lam_k, V, m, lam)
    # sqrt(lambda) phi(P_q) = sqrt(lambda) v_q / sqrt(w)
    np.testing.assert_allclose(B, (np.sqrt(lam_k)[:, None] * V.T) * m, atol=1e-12)


def test_extended_functions_are_orthonormal():
    # the Nystrom extensions are orthogonal in L2(D) up to the quadrature
    # error; at the elements' centroids of a fine level (equal-area
    # weights) the Gram matrix of B / sqrt(lambda) is close to I
    m, lam, l = 24, 0.65, 6
    lam_k, V, _ = matern.modes(6, m, lam)
    X = matern.centroids(l)
    B = matern.extend(X, lam_k, V, m, lam) / np.sqrt(lam_k)[:, None]
    G = B @ B.T / X.shape[0]
    np.testing.assert_allclose(G, np.eye(6), atol=5e-3)


def test_centroids_match_the_fem_oracle():
    for l in (1, 2, 4):
        np.testing.assert_array_equal(matern.centroids(l), oracle.centroids(l))
