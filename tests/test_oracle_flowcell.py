"""Pins of the flow-cell oracle (Sec. 5, Example 5.3: p = 0 at x1 = 0, p = 1 at
x1 = 1, no flow through x2 = 0 and x2 = 1, no source).

Exact cases the P1 solution must reproduce: a coefficient constant in each
row of cells gives p = x1; one constant in each column of cells gives the
1-D harmonic profile; the discrete flux is conserved; the discrete maximum
principle holds (right triangles give an M-matrix); the observation of a
linear field is the field at the point.  A dropped Neumann row, a wrong
Dirichlet lift or a transposed element would break one of them.
"""
import numpy as np
import pytest

from oracle import flowcell as fc
from tests import inputs


def _rows_of_cells(l, vals):
    n = 1 << l
    j = (np.arange(2 * n * n) // 2) // n
    return vals[j]


def _cols_of_cells(l, vals):
    n = 1 << l
    i = (np.arange(2 * n * n) // 2) % n
    return vals[i]


@pytest.mark.parametrize("l", [1, 2, 4])
def test_constant_and_layered_coefficients_give_linear_pressure(l):
    n = 1 << l
    xy = fc.node_xy(l)
    for kap in (np.full(2 * n * n, 3.7), _rows_of_cells(l, np.exp(np.random.default_rng(l).normal(size=n)))):
        p = fc.solve_nodes(l, kap)
        np.testing.assert_allclose(p, xy[:, 0], atol=1e-12)
    m = 5
    G = fc.forward_kappa(l, m, np.full(2 * n * n, 0.3))[0]
    a = np.tile(np.arange(1, m + 1), m) / (m + 1)
    np.testing.assert_allclose(G, a, atol=1e-12)


@pytest.mark.parametrize("l", [2, 3, 5])
def test_column_coefficients_give_the_harmonic_profile(l):
    n = 1 << l
    kc = np.exp(np.random.default_rng(10 + l).normal(size=n))
    p = fc.solve_nodes(l, _cols_of_cells(l, kc)).reshape(n + 1, n + 1)
    prof = np.concatenate([[0.0], np.cumsum(1.0 / kc)]) / np.sum(1.0 / kc)
    np.testing.assert_allclose(p, np.tile(prof, (n + 1, 1)), atol=1e-12)


def test_flux_is_conserved_and_maximum_principle_holds():
    l = 4
    n = 1 << l
    kap = inputs.kappa_batch(3, 1, 2 * n * n, spread=1.5)[0]
    A = fc.assemble(l, kap)
    p = fc.solve_nodes(l, kap)
    r = (A @ p).reshape(n + 1, n + 1)
    assert np.abs(r[:, 1:n]).max() < 1e-12          # the equation at every unknown
    assert abs(r[:, 0].sum() + r[:, n].sum()) < 1e-12  # inflow = outflow
    assert r[:, n].sum() > 0
    assert p.min() >= -1e-14 and p.max() <= 1 + 1e-14
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12  # natural BCs: constants in the kernel


def test_unknown_ordering_and_sizes():
    l = 3
    n = 1 << l
    assert fc.n_unknowns(l) == (n - 1) * (n + 1)
    p = np.arange((n + 1) ** 2, dtype=float)
    u = fc.unknowns_of(l, p)
    assert u[0] == 1 and u[n - 2] == n - 1 and u[n - 1] == (n + 1) + 1
    assert u.size == fc.n_unknowns(l)


def test_second_order_convergence_at_the_nodes():
    # smooth coefficient kappa(x) = exp(sin(2 pi x1) cos(pi x2)) at the centroids
    def kap(l):
        n = 1 << l
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
        i, j = i.ravel(), j.ravel()
        c = np.zeros((2 * n * n, 2))
        c[0::2] = np.stack([(3 * i + 2) / (3 * n), (3 * j + 1) / (3 * n)], 1)
        c[1::2] = np.stack([(3 * i + 1) / (3 * n), (3 * j + 2) / (3 * n)], 1)
        return np.exp(np.sin(2 * np.pi * c[:, 0]) * np.cos(np.pi * c[:, 1]))
    ref = fc.solve_nodes(7, kap(7)).reshape(129, 129)
    errs = []
    for l in (3, 4, 5):
        n = 1 << l
        p = fc.solve_nodes(l, kap(l)).reshape(n + 1, n + 1)
        st = 128 // n
        errs.append(np.abs(p - ref[::st, ::st]).max())
    assert errs[1] < 0.35 * errs[0] and errs[2] < 0.35 * errs[1]


@pytest.mark.parametrize("l", [1, 3, 5])
def test_sampler_flow_model_reproduces_the_exact_cases(l):
    """The sampler's own flow-cell forward (compiled, banded Cholesky) on the
    same exact cases: p = x1 for coefficients constant in each row of cells,
    the harmonic profile for coefficients constant in each column, and the
    observation of p = x1 is the first coordinate of each point."""
    import oracle
    n, m = 1 << l, 5
    xy = fc.node_xy(l)
    lay = _rows_of_cells(l, np.exp(np.random.default_rng(20 + l).normal(size=n)))
    G, p = oracle.flow_forward_kappa(l, m, lay[None], want_p=True)
    np.testing.assert_allclose(p[0], fc.unknowns_of(l, xy[:, 0]), atol=1e-12)
    np.testing.assert_allclose(G[0], np.tile(np.arange(1, m + 1), m) / (m + 1), atol=1e-12)
    kc = np.exp(np.random.default_rng(30 + l).normal(size=n))
    prof = np.concatenate([[0.0], np.cumsum(1.0 / kc)]) / np.sum(1.0 / kc)
    G, p = oracle.flow_forward_kappa(l, m, _cols_of_cells(l, kc)[None], want_p=True)
    np.testing.assert_allclose(p[0], fc.unknowns_of(l, np.tile(prof, n + 1)), atol=1e-12)


def test_sampler_flow_model_matches_the_sparse_flow_oracle():
    import oracle
    for l in (2, 4, 6):
        kap = inputs.kappa_batch(40 + l, 3, 2 * 4 ** l, spread=1.0)
        G, p = oracle.flow_forward_kappa(l, 7, kap, want_p=True)
        Gr, pr = fc.forward_kappa(l, 7, kap, want_p=True)
        assert np.abs(G - Gr).max() < 1e-12 and np.abs(p - pr).max() < 1e-12
