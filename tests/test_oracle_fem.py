"""Pins of the oracle's P1 finite-element forward model (Sec. 5):
-div(kappa grad p) = f on (0,1)^2, p = 0 on the boundary, uniform meshes of
2 n^2 triangles, point observations.
"""
import numpy as np
import pytest

import oracle
from tests import inputs


def _interior_xy(l):
    n = 1 << l
    ii, jj = np.meshgrid(np.arange(1, n), np.arange(1, n))
    return ii.ravel() / n, jj.ravel() / n


def _band_matvec(l, band, x):
    n = 1 << l
    M = len(x)
    y = band[:, 0] * x
    for k in range(1, n + 1):
        y[k:] += band[k:, k] * x[:-k]
        y[:-k] += band[k:, k] * x[k:]
    return y


def _torsion(x, y, terms=60):
    """exact solution of -Lap p = 1, p = 0 on the boundary of the unit square"""
    s = x * (1 - x) / 2
    for m in range(1, 2 * terms, 2):
        s = s - 4 / (np.pi ** 3 * m ** 3) * np.sin(m * np.pi * x) * np.cosh(m * np.pi * (y - 0.5)) / np.cosh(m * np.pi / 2)
    return s


@pytest.mark.parametrize("l", [2, 3, 4, 5, 6, 7])
def test_manufactured_quadratic_is_nodally_exact(l):
    # kappa = 1, p = x(1-x)y(1-y), nodal load h^2 f(x_u): the operator is exact
    # on products of quadratics, so the discrete solution equals p at nodes
    x, y = _interior_xy(l)
    f = 2 * (x * (1 - x) + y * (1 - y))
    p = oracle.solve(l, np.ones(oracle.n_elem(l)), oracle.load(l, f))
    assert np.abs(p - x * (1 - x) * y * (1 - y)).max() < 1e-13 * 4 ** (l - 2)


def test_torsion_series_cross_check():
    x, y = np.array([0.3, 0.5, 0.71]), np.array([0.2, 0.5, 0.9])
    M = 301
    m = np.arange(1, M, 2)[:, None, None]
    k = np.arange(1, M, 2)[None, :, None]
    ds = (16 * np.sin(m * np.pi * x) * np.sin(k * np.pi * y) / (np.pi ** 4 * m * k * (m ** 2 + k ** 2))).sum((0, 1))
    np.testing.assert_allclose(_torsion(x, y), ds, atol=2e-6)


def test_torsion_convergence_rate():
    errs = []
    levels = [3, 4, 5, 6, 7]
    for l in levels:
        x, y = _interior_xy(l)
        p = oracle.solve(l, np.ones(oracle.n_elem(l)), oracle.load(l))
        errs.append(np.sqrt(np.mean((p - _torsion(x, y)) ** 2)))
    slope = -np.polyfit(levels, np.log2(errs), 1)[0]
    assert abs(slope - 2) < 0.1, (errs, slope)


def test_observations_converge_to_torsion():
    m = 5
    pts = [(a / (m + 1), b / (m + 1)) for b in range(1, m + 1) for a in range(1, m + 1)]
    ex = np.array([_torsion(px, py) for px, py in pts])
    e = []
    for l in [4, 5, 6, 7]:
        p = oracle.solve(l, np.ones(oracle.n_elem(l)), oracle.load(l))
        e.append(np.abs(oracle.observe(l, m, p) - ex).max())
    r = np.array(e[:-1]) / np.array(e[1:])
    assert np.all(r > 3.0), e


@pytest.mark.parametrize("l", [3, 4])
@pytest.mark.parametrize("ab", [(1, 1), (2, 3), (5, 1)])
def test_sine_mode_eigenpairs(l, ab):
    a, b = ab
    n = 1 << l
    h = 1.0 / n
    c = 2.5
    x, y = _interior_xy(l)
    v = np.sin(a * np.pi * x) * np.sin(b * np.pi * y)
    band = oracle.assemble_band(l, c * np.ones(oracle.n_elem(l)))
    lam = c * (4 * np.sin(a * np.pi * h / 2) ** 2 + 4 * np.sin(b * np.pi * h / 2) ** 2)
    np.testing.assert_allclose(_band_matvec(l, band, v), lam * v, atol=1e-13)


def test_dense_symmetric_spd_and_row_sums():
    l = 3
    n = 1 << l
    kap = inputs.kappa_batch(1, 1, oracle.n_elem(l))[0]
    A = oracle.assemble_dense(l, kap)
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    rng = inputs.rng(2)
    for _ in range(5):
        z = rng.standard_normal(A.shape[0])
        assert z @ A @ z > 0
    # rows of nodes whose four neighbours are interior sum to zero
    for j in range(2, n - 1):
        for i in range(2, n - 1):
            u = (j - 1) * (n - 1) + (i - 1)
            assert abs(A[u].sum()) < 1e-13 * A[u, u]


def test_generic_assembly_is_five_point_edge_formula():
    # with the SW-NE diagonal each triangle is right-angled; the hypotenuse
    # coupling vanishes and each leg carries -(kappa_T1 + kappa_T2)/2
    l = 3
    n = 1 << l
    kap = inputs.kappa_batch(4, 1, oracle.n_elem(l))[0]
    A = oracle.assemble_dense(l, kap)

    def k(i, j, t):
        return kap[2 * (j * n + i) + t]

    def unk(i, j):
        return (j - 1) * (n - 1) + (i - 1) if 1 <= i <= n - 1 and 1 <= j <= n - 1 else None

    ref = np.zeros_like(A)
    edges = []
    for j in range(n + 1):
        for i in range(n):  # horizontal edge (i,j)-(i+1,j): lower tri of cell (i,j), upper of (i,j-1)
            w = (k(i, j, 0) if j < n else 0) + (k(i, j - 1, 1) if j > 0 else 0)
            edges.append(((i, j), (i + 1, j), w / 2))
    for j in range(n):
        for i in range(n + 1):  # vertical edge (i,j)-(i,j+1): upper tri of cell (i,j), lower of (i-1,j)
            w = (k(i, j, 1) if i < n else 0) + (k(i - 1, j, 0) if i > 0 else 0)
            edges.append(((i, j), (i, j + 1), w / 2))
    for a, b, w in edges:
        ua, ub = unk(*a), unk(*b)
        if ua is not None:
            ref[ua, ua] += w
        if ub is not None:
            ref[ub, ub] += w
        if ua is not None and ub is not None:
            ref[ua, ub] -= w
            ref[ub, ua] -= w
    np.testing.assert_allclose(A, ref, rtol=1e-14, atol=1e-14)


def test_band_matches_dense_and_reciprocity():
    l = 4
    kap = inputs.kappa_batch(5, 1, oracle.n_elem(l), spread=1.5)[0]
    A = oracle.assemble_dense(l, kap)
    band = oracle.assemble_band(l, kap)
    x = inputs.rng(6).standard_normal(A.shape[0])
    np.testing.assert_allclose(_band_matvec(l, band, x), A @ x, rtol=1e-13, atol=1e-13)
    ea = np.zeros(A.shape[0]); ea[17] = 1
    eb = np.zeros(A.shape[0]); eb[150] = 1
    pa = oracle.solve(l, kap, ea)
    pb = oracle.solve(l, kap, eb)
    assert abs(pa[150] - pb[17]) < 1e-14 * abs(pa[150]) + 1e-18


def test_tiny_meshes():
    # l = 1: one unknown at (1/2,1/2); load h^2 = 1/4 (f = 1 exactly)
    kap = np.array([0.5, 2.0, 1.5, 3.0, 0.7, 1.1, 2.2, 0.9])
    A = oracle.assemble_dense(1, kap)
    assert A.shape == (1, 1)
    # the six triangles at the centre: a right angle there contributes kappa
    # (elements 3 and 4), an acute angle kappa/2 (elements 0, 1, 6, 7)
    ref = (kap[0] / 2 + kap[1] / 2 + kap[3] + kap[4] + kap[6] / 2 + kap[7] / 2)
    assert abs(A[0, 0] - ref) < 1e-15
    p = oracle.solve(1, kap, oracle.load(1))
    assert abs(p[0] - 0.25 / ref) < 1e-16
    # l = 2: 9 unknowns against a dense solve
    kap2 = inputs.kappa_batch(8, 1, oracle.n_elem(2))[0]
    A2 = oracle.assemble_dense(2, kap2)
    b2 = oracle.load(2)
    np.testing.assert_allclose(oracle.solve(2, kap2, b2), np.linalg.solve(A2, b2), rtol=1e-14)


def test_load_f_one_is_h_squared():
    for l in [1, 3, 6]:
        np.testing.assert_allclose(oracle.load(l), (0.5 ** l) ** 2 * np.ones(oracle.n_unknowns(l)), rtol=1e-15)


@pytest.mark.parametrize("l", [2, 4, 6])
def test_observation_nodal_and_linear_exactness(l):
    n = 1 << l
    x, y = _interior_xy(l)
    # m = 3: points a/4 are nodes for l >= 2
    p = np.sin(3 * x) + y ** 2
    G = oracle.observe(l, 3, p)
    for b in range(1, 4):
        for a in range(1, 4):
            assert G[(b - 1) * 3 + (a - 1)] == p[(b * n // 4 - 1) * (n - 1) + (a * n // 4 - 1)]
    # a linear field vanishing on the boundary does not exist, so use a field
    # whose boundary values are zero only where needed: check at points inside
    # the band of cells away from the boundary, for m = 5, 7, 10
    for m in [5, 7, 10]:
        lin = 0.3 + 1.7 * x - 0.9 * y
        G = oracle.observe(l, m, lin)
        pts = [(a / (m + 1), b / (m + 1)) for b in range(1, m + 1) for a in range(1, m + 1)]
        for o, (px, py) in enumerate(pts):
            if min(px, py) > 1.0 / n and max(px, py) < 1 - 1.0 / n:
                assert abs(G[o] - (0.3 + 1.7 * px - 0.9 * py)) < 1e-13


def test_potential_definition():
    G = np.array([0.1, 0.2, 0.4])
    y = np.array([0.0, 0.3, 0.2])
    assert abs(oracle.potential(G, y, 0.1) - 0.5 * ((0.1 ** 2 + 0.1 ** 2 + 0.2 ** 2) / 0.01)) < 1e-13


def test_forward_batch_equals_single_solves():
    l, K, m = 3, 5, 3
    th = inputs.theta_batch(9, 4, K)
    G = oracle.forward(l, K, 1.0, 0.3, m, th, nthreads=2)
    B = oracle.kl_basis(l, K, 1.0, 0.3)
    for q in range(4):
        p = oracle.solve(l, np.exp(th[q] @ B), oracle.load(l))
        np.testing.assert_allclose(G[q], oracle.observe(l, m, p), rtol=1e-14)


@pytest.mark.parametrize("l", [2, 3, 5])
@pytest.mark.parametrize("m", [5, 7, 10])
def test_observation_barycentric_on_containing_triangle(l, m):
    # a random nodal field is not linear across the cell diagonal, so the value
    # at each point must come from the triangle that contains the point; the
    # barycentric coordinates are found here by a generic 3x3 solve
    n = 1 << l
    p = inputs.rng(l * 100 + m).standard_normal(oracle.n_unknowns(l))
    G = oracle.observe(l, m, p)

    def nodal(i, j):
        if 1 <= i <= n - 1 and 1 <= j <= n - 1:
            return p[(j - 1) * (n - 1) + (i - 1)]
        return 0.0

    for b in range(1, m + 1):
        for a in range(1, m + 1):
            x, y = a / (m + 1), b / (m + 1)
            i, j = min(int(np.floor(x * n)), n - 1), min(int(np.floor(y * n)), n - 1)
            lo = [(i, j), (i + 1, j), (i + 1, j + 1)]
            up = [(i, j), (i + 1, j + 1), (i, j + 1)]
            vals = None
            for tri in (lo, up):
                V = np.array([[vi / n, vj / n, 1.0] for vi, vj in tri]).T
                lam = np.linalg.solve(V, np.array([x, y, 1.0]))
                if np.all(lam >= -1e-12):
                    vals = sum(lm * nodal(*v) for lm, v in zip(lam, tri))
                    break
            assert vals is not None
            assert abs(G[(b - 1) * m + (a - 1)] - vals) < 1e-12
