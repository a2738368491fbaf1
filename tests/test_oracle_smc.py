"""Pins of the oracle's adaptive step (Sec. 3.4) and resampling (Sec. 2.4)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import inputs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kish_identity(seed):
    d = inputs.potentials(seed, 500)
    for t in [1e-4, 1e-2, 0.3]:
        w = np.exp(-t * d)
        cv2 = w.var() / w.mean() ** 2  # population variance
        assert abs(oracle.ess(d, 1.0, t) - 500 / (1 + cv2)) < 1e-10 * 500


def test_ess_monotone_in_t():
    d = inputs.potentials(3, 300)
    ts = np.linspace(0, 1, 200)
    e = np.array([oracle.ess(d, 0.7, t) for t in ts])
    assert np.all(np.diff(e) <= 1e-12)
    assert abs(e[0] - 300) < 1e-9


def test_uniform_potential_takes_full_step():
    d = np.full(100, 3.7)
    r = oracle.next_step(d, 1.0, 0.25, 50.0)
    assert r["next"] == 1.0
    np.testing.assert_allclose(r["w"], 0.01, rtol=1e-14)
    assert abs(r["dlogZ"] - (-0.75 * 3.7)) < 1e-12


def test_one_dominant_particle_takes_minimum_step():
    d = np.zeros(100)
    d[1:] = 1e9
    r = oracle.next_step(d, 1.0, 0.0, 50.0, eps=1e-6)
    assert r["next"] == 1e-6
    assert r["ess"] < 1.0 + 1e-9


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_interior_root_and_argmin(seed):
    d = inputs.potentials(seed, 400, scale=50.0)
    tau = 200.0
    r = oracle.next_step(d, 1.0, 0.0, tau)
    t = r["next"]
    assert 1e-6 < t < 1
    assert abs(oracle.ess(d, 1.0, t) - tau) < 1e-9 * 400
    assert oracle.ess(d, 1.0, t) >= tau
    # argmin of (ESS - tau)^2 against a brute-force grid
    grid = np.linspace(1e-6, 1, 4001)
    obj = np.array([(oracle.ess(d, 1.0, g) - tau) ** 2 for g in grid])
    assert (oracle.ess(d, 1.0, t) - tau) ** 2 <= obj.min() + 1e-12
    # weights: normalised, proportional to exp(-t d), evidence increment
    w_ref = np.exp(-t * (d - d.min()))
    np.testing.assert_allclose(r["w"], w_ref / w_ref.sum(), rtol=1e-12)
    assert abs(r["dlogZ"] - np.log(np.mean(np.exp(-t * d)))) < 1e-10


def test_bridging_scale_and_offset():
    # bridging: lw = -(zeta'-zeta) * beta * (Phi_hi - Phi_lo), starting at zeta
    d = inputs.potentials(7, 300, scale=5.0) - 10.0
    beta, zeta = 0.4, 0.3
    r = oracle.next_step(d, beta, zeta, 150.0)
    t = r["next"] - zeta
    assert r["next"] <= 1.0
    np.testing.assert_allclose(r["logw"], -t * beta * d, rtol=1e-12, atol=1e-12)
    if r["next"] < 1.0:
        assert abs(oracle.ess(d, beta, t) - 150.0) < 1e-6


def test_next_step_rejects_nonfinite():
    d = np.ones(10)
    d[3] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.next_step(d, 1.0, 0.0, 5.0)


def _exact_ancestors(w, u):
    """inverse CDF on exact rationals: a_i = min{j : sum_{k<=j} w_k > u_i W}"""
    W = sum(Fraction(x) for x in w)
    out = []
    for ui in u:
        acc = Fraction(0)
        for j, x in enumerate(w):
            acc += Fraction(x)
            if acc > Fraction(ui) * W:
                out.append(j)
                break
    return np.array(out)


@pytest.mark.parametrize("J", [1, 2, 3, 4])
def test_resample_brute_force_exact(J):
    rng = inputs.rng(J)
    for trial in range(30):
        # dyadic weights with few bits, so quantisation is exact
        w = rng.integers(0, 17, size=J).astype(float) / 16.0
        if w.max() == 0:
            w[0] = 1.0
        u = np.arange(64) / 64.0
        # every grid uniform, in chunks of J (one uniform per particle)
        for start in range(0, 64, J):
            uu = u[start:start + J]
            if len(uu) < J:
                break
            anc = oracle.resample(w, uu)
            np.testing.assert_array_equal(anc, _exact_ancestors(w, uu))


def test_resample_zero_weights_never_drawn_and_order():
    w = inputs.weights(3, 1000, zero_frac=0.3)
    u = inputs.uniforms53(4, 1000)
    anc = oracle.resample(w, u)
    assert np.all(w[anc] > 0)
    # order of outputs follows i: same u value -> same ancestor, and ancestors
    # are monotone in u
    o = np.argsort(u, kind="stable")
    assert np.all(np.diff(anc[o]) >= 0)


def test_resample_chi_square():
    J = 20000
    w = np.linspace(1.0, 3.0, 8)
    w = np.resize(w, J) * (np.arange(J) < 8)  # only the first 8 particles carry weight
    u = inputs.uniforms53(5, J)
    anc = oracle.resample(w, u)
    counts = np.bincount(anc, minlength=8)[:8]
    p = w[:8] / w[:8].sum()
    chi2 = ((counts - J * p) ** 2 / (J * p)).sum()
    assert counts.sum() == J
    assert chi2 < 24.3  # chi^2_7 upper 0.1 % point


def test_resample_invariant_to_weight_scale():
    w = inputs.weights(6, 333)
    u = inputs.uniforms53(7, 333)
    a1 = oracle.resample(w, u)
    a2 = oracle.resample(w * 2.0 ** 40, u)
    np.testing.assert_array_equal(a1, a2)


def test_resample_rejects_bad_input():
    with pytest.raises(oracle.OracleError):
        oracle.resample(np.zeros(4), np.zeros(4))
    with pytest.raises(oracle.OracleError):
        oracle.resample(np.array([1.0, -1.0]), np.zeros(2))


def test_pcn_proposal_and_acceptance_rule():
    th = inputs.theta_batch(1, 5, 3)
    xi = inputs.theta_batch(2, 5, 3)
    out = oracle.pcn_propose(th, xi, 0.5)
    np.testing.assert_allclose(out, np.sqrt(0.75) * th + 0.5 * xi, rtol=1e-15)
    assert oracle.mh_accept(1.0, 0.5, 0.999)  # downhill always
    assert not oracle.mh_accept(0.0, 50.0, 0.5)
    u = 0.3
    assert oracle.mh_accept(0.0, -np.log(u) - 1e-9, u)
    assert not oracle.mh_accept(0.0, -np.log(u) + 1e-9, u)
