"""GPU sampler on the linear test model G_l(theta) = (A + 2^{-2l} E) theta
(Sec. 2.1 with a linear forward map), and the exported look-ahead statistic
of the level-update test (Sec. 4.4).

* the look-ahead ESS and cv^2 equal the oracle's ESS at t = 1;
* with the linear model in place of the PDE, single pCN steps and whole
  MLS^2MC runs (tempering, bridging, look-ahead, multilevel bridging) equal
  the oracle's on the same Philox streams, stage for stage;
* the GPU sampler reproduces the closed-form Gaussian posterior mean and
  variance and the evidence within 4 Monte Carlo standard errors over 20
  seeds, on one level and over four levels with bridging, and so does the
  delayed-acceptance form with the GPU-trained network (the two-stage rule
  is exact for any surrogate).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1709_09763_amd as P
from tests import inputs
from tests.gpu_util import case, device, host, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _lin_problem(K=3, nobs=4, s=0.2, seed=0):
    g = inputs.rng(seed)
    A = g.standard_normal((nobs, K))
    E = g.standard_normal((nobs, K))
    th = g.standard_normal(K)
    y = A @ th + s * g.standard_normal(nobs)
    return A, E, y


def _lin_posterior(A, y, s):
    """N(0, I) prior, y = A theta + N(0, s^2 I): posterior N(m, C) and the
    log-evidence of the unnormalised likelihood exp(-|y - A theta|^2 / 2s^2)"""
    K = A.shape[1]
    Pm = np.eye(K) + A.T @ A / s ** 2
    C = np.linalg.inv(Pm)
    m = C @ A.T @ y / s ** 2
    # Z = (2 pi s^2)^{nobs/2} N(y; 0, G) with G = s^2 I + A A^T, and
    # det G = s^{2 nobs} det Pm
    G = s ** 2 * np.eye(len(y)) + A @ A.T
    logZ = -0.5 * np.linalg.slogdet(Pm)[1] - 0.5 * y @ np.linalg.solve(G, y)
    return m, C, logZ


@pytest.mark.parametrize("N,scale", [(100, 0.3), (1000, 1.0), (4099, 0.02)])
def test_cv_lu_matches_oracle_ess(N, scale):
    device()
    case(f"cv_lu N={N}")
    c = P.Context(3, 4, 5, 1.0, 0.3, 2, 0.1)
    d = inputs.potentials(70 + N, N, scale=40.0) - 30.0
    out = host(c.cv_lu(to_dev(d), scale))
    ess = oracle.ess(d, scale, 1.0)
    assert abs(out[0] - ess) <= 1e-12 * ess
    assert abs(out[1] - (N / ess - 1.0)) <= 1e-10 * max(1.0, N / ess)
    # uniform weights: cv = 0
    out = host(c.cv_lu(to_dev(np.full(N, 3.25)), scale))
    assert out[0] == pytest.approx(N, rel=1e-14) and abs(out[1]) < 1e-12
    d[N // 2] = np.inf
    assert np.isnan(host(c.cv_lu(to_dev(d), scale))).all()


def test_linear_forward_and_pcn_step_match_oracle_rule():
    device()
    case("linear model forward + pcn_step")
    K, N, sn = 3, 400, 0.2
    A, E, y = _lin_problem(K=K, s=sn, seed=1)
    c = P.Context(2, 5, K, 1.0, 0.3, 2, sn)
    c.set_linear_model(A, 7.0 * E)
    th = inputs.theta_batch(2, N, K)
    for l in (2, 5):
        G = host(c.forward(l, to_dev(th)))
        assert rel_err(G, th @ (A + 2.0 ** (-2 * l) * 7.0 * E).T) < 1e-14
    l_lo, l_hi, beta, zeta = 3, 4, 0.4, 0.3
    Gm = {l: th @ (A + 2.0 ** (-2 * l) * 7.0 * E).T for l in (l_lo, l_hi)}
    ph = {l: np.array([oracle.potential(g, y, sn) for g in Gm[l]]) for l in (l_lo, l_hi)}
    xi = inputs.theta_batch(3, N, K)
    u = 1.0 - inputs.uniforms53(4, N)
    thp = oracle.pcn_propose(th, xi, 0.5)
    php = {l: np.array([oracle.potential(g, y, sn) for g in thp @ (A + 2.0 ** (-2 * l) * 7.0 * E).T])
           for l in (l_lo, l_hi)}
    old = beta * ((1 - zeta) * ph[l_lo] + zeta * ph[l_hi])
    new = beta * ((1 - zeta) * php[l_lo] + zeta * php[l_hi])
    acc_ref = np.array([oracle.mh_accept(o, n_, uu) for o, n_, uu in zip(old, new, u)])
    T = to_dev(th)
    acc = host(c.pcn_step(l_lo, l_hi, beta, zeta, 0.5, T, to_dev(Gm[l_lo]), to_dev(Gm[l_hi]),
                          to_dev(ph[l_lo]), to_dev(ph[l_hi]), to_dev(y), to_dev(xi), to_dev(u)))
    np.testing.assert_array_equal(acc.astype(bool), acc_ref)
    assert 0 < acc_ref.sum() < N
    assert rel_err(host(T), np.where(acc_ref[:, None], thp, th)) < 1e-15
    # the PDE comes back when the model is cleared
    c.set_linear_model(None, None)
    G, st, _ = c.forward(3, to_dev(th[:8]), with_stats=True)
    assert (host(st) == 0).all()
    assert rel_err(host(G), oracle.forward(3, K, 1.0, 0.3, 2, th[:8])) < 1e-10


def test_linear_model_rejected_by_batched_and_field_calls():
    device()
    c = P.Context(2, 3, 3, 1.0, 0.3, 2, 0.2)
    A, E, _ = _lin_problem()
    c.set_linear_model(A, E)
    with pytest.raises(P.Mls2mcError, match="linear test model"):
        c.forward_field(2, torch.ones((1, 32), dtype=torch.float64, device="cuda:0"))
    with pytest.raises(P.Mls2mcError, match="linear test model"):
        G = torch.empty((1, 4), dtype=torch.float64, device="cuda:0")
        P.mls2mc_forward_batch(c.h, [dict(l=2, theta=to_dev(np.zeros((1, 3))), G_out=G)])


@pytest.mark.parametrize("cfg", [
    dict(name="single level", l_min=3, l_max=3, dep=1.0, scheme=0),
    dict(name="MLS2MC 4 levels", l_min=2, l_max=5, dep=30.0, scheme=0),
    dict(name="multilevel bridging", l_min=2, l_max=5, dep=3.0, scheme=1),
    dict(name="adaptive maximum level", l_min=1, l_max=4, dep=0.0, scheme=0, tau_min=1e-3),
])
def test_linear_run_matches_oracle(cfg):
    device()
    case(f"linear run {cfg['name']}")
    s, J = 0.15, 1000
    A, E, y = _lin_problem(K=2, nobs=4, s=s, seed=3)
    E = cfg["dep"] * E
    c = P.Context(cfg["l_min"], cfg["l_max"], 2, 1.0, 0.3, 2, s)
    c.set_linear_model(A, E)
    kw = dict(scheme=cfg["scheme"], tau_min=cfg.get("tau_min", 0.0))
    g = c.run(to_dev(y), J, J_tilde=100, seed=7, **kw)
    r = oracle.run_sampler(y, model="linear", l_min=cfg["l_min"], l_max=cfg["l_max"], K=2, nobs=4, sigma_n=s,
                           J=J, J_tilde=100, seed=7, lin_A=A, lin_E=E, **kw)
    print(f"  stages {g['n_stages']} / {r['n_stages']}, final level {g['final_level']}")
    assert g["n_stages"] == r["n_stages"] and g["final_level"] == r["final_level"]
    np.testing.assert_array_equal(g["stage_type"], r["stage_type"])
    np.testing.assert_array_equal(g["stage_level"], r["stage_level"])
    np.testing.assert_allclose(g["stage_beta"], r["stage_beta"], rtol=1e-12)
    np.testing.assert_allclose(g["stage_zeta"], r["stage_zeta"], rtol=1e-12, atol=1e-15)
    assert g["solves"] == r["solves"]
    assert g["accepted"] == r["accepted"]
    assert abs(g["log_Z"] - r["log_Z"]) < 1e-10 * max(1, abs(r["log_Z"]))
    assert rel_err(host(g["theta"]), r["theta"]) < 1e-12
    if cfg.get("tau_min"):
        assert g["final_level"] == 1  # identical levels: u' stops on the coarsest one


@pytest.mark.parametrize("cfg", [
    dict(name="single level", l_min=3, l_max=3, dep=1.0, scheme=0),
    dict(name="MLS2MC 4 levels", l_min=2, l_max=5, dep=30.0, scheme=0),
    dict(name="multilevel bridging", l_min=2, l_max=5, dep=3.0, scheme=1),
])
def test_linear_delayed_acceptance_run_matches_oracle(cfg):
    """Whole delayed-acceptance runs: a linear surrogate G~ = S theta screens
    every pCN move (tempering and bridging, from the coarsest level on), the
    linear model judges the survivors.  Stage for stage the same stage types,
    levels, steps, first-stage passes and acceptances as the oracle's
    sampler with the same surrogate, the same evidence and particles.  (The
    oracle evaluates every proposal, the library only the survivors, so
    their solve counts differ by design.)"""
    device()
    case(f"linear delayed-acceptance run {cfg['name']}")
    s, J = 0.15, 1000
    A, E, y = _lin_problem(K=2, nobs=4, s=s, seed=3)
    E = cfg["dep"] * E
    S = A + 0.3 * inputs.rng(31).standard_normal(A.shape)  # a surrogate that is off by a fair margin
    c = P.Context(cfg["l_min"], cfg["l_max"], 2, 1.0, 0.3, 2, s)
    c.set_linear_model(A, E)
    c.set_linear_surrogate(S)
    kw = dict(scheme=cfg["scheme"])
    g = c.run(to_dev(y), J, J_tilde=100, seed=9, surrogate=True, sur_da_min_level=cfg["l_min"], **kw)
    r = oracle.run_sampler(y, model="linear", l_min=cfg["l_min"], l_max=cfg["l_max"], K=2, nobs=4, sigma_n=s,
                           J=J, J_tilde=100, seed=9, lin_A=A, lin_E=E, da_S=S, **kw)
    print(f"  stages {g['n_stages']} / {r['n_stages']}, stage-1 passes {g['stage1_passed']} / "
          f"{r['stage1_passed']} of {g['da_proposed']}, accepted {g['accepted']} / {r['accepted']}")
    assert g["n_stages"] == r["n_stages"] and g["final_level"] == r["final_level"]
    np.testing.assert_array_equal(g["stage_type"], r["stage_type"])
    np.testing.assert_array_equal(g["stage_level"], r["stage_level"])
    np.testing.assert_allclose(g["stage_beta"], r["stage_beta"], rtol=1e-12)
    np.testing.assert_allclose(g["stage_zeta"], r["stage_zeta"], rtol=1e-12, atol=1e-15)
    assert g["da_proposed"] == g["proposed"] == r["proposed"]  # every move was screened
    assert g["stage1_passed"] == r["stage1_passed"] and 0 < g["stage1_passed"] < g["da_proposed"]
    assert g["accepted"] == r["accepted"]
    assert abs(g["log_Z"] - r["log_Z"]) < 1e-10 * max(1, abs(r["log_Z"]))
    assert rel_err(host(g["theta"]), r["theta"]) < 1e-12
    assert g["sur_err_count"] == g["stage1_passed"] and g["sur_err_mean"] > 0
    c.set_linear_surrogate(None)
    c.set_linear_model()


def _closed_form_check(runs, m, C, logZ, R):
    means = np.array([host(r["theta"]).mean(0) for r in runs])
    vars_ = np.array([host(r["theta"]).var(0) for r in runs])
    lz = np.array([r["log_Z"] for r in runs])
    se = means.std(0, ddof=1) / np.sqrt(R)
    print(f"  mean {means.mean(0)} vs {m}; var {vars_.mean(0)} vs {np.diag(C)}; "
          f"log Z {lz.mean():.4f} +- {lz.std(ddof=1) / np.sqrt(R):.4f} vs {logZ:.4f}")
    assert np.all(np.abs(means.mean(0) - m) < 4 * se + 0.02 * np.sqrt(np.diag(C)))
    np.testing.assert_allclose(vars_.mean(0), np.diag(C), rtol=0.1)
    assert abs(lz.mean() - logZ) < 4 * lz.std(ddof=1) / np.sqrt(R) + 0.05


def test_linear_gaussian_posterior_single_level():
    device()
    case("linear-Gaussian closed form, one level, 20 seeds")
    s, R, J = 0.2, 20, 2000
    A, E, y = _lin_problem(s=s)
    m, C, logZ = _lin_posterior(A + 2.0 ** -6 * E, y, s)
    c = P.Context(3, 3, 3, 1.0, 0.3, 2, s)
    c.set_linear_model(A, E)
    runs = [c.run(to_dev(y), J, seed=seed) for seed in range(R)]
    assert all(np.all(r["stage_type"] == 0) for r in runs)
    _closed_form_check(runs, m, C, logZ, R)


def test_linear_gaussian_posterior_multilevel():
    device()
    case("linear-Gaussian closed form, 4 levels with bridging, 20 seeds")
    s, R, J = 0.15, 20, 2000
    A, E, y = _lin_problem(K=2, nobs=4, s=s, seed=3)
    E = 30.0 * E
    m, C, logZ = _lin_posterior(A + 2.0 ** -10 * E, y, s)
    c = P.Context(2, 5, 2, 1.0, 0.3, 2, s)
    c.set_linear_model(A, E)
    runs = [c.run(to_dev(y), J, J_tilde=100, seed=100 + seed) for seed in range(R)]
    kinds = set()
    for r in runs:
        assert r["final_level"] == 5 and r["final_beta"] == 1.0
        kinds |= set(r["stage_type"].tolist())
    assert 0 in kinds and (2 in kinds or 3 in kinds)
    _closed_form_check(runs, m, C, logZ, R)


def test_linear_gaussian_posterior_with_delayed_acceptance():
    """The network, trained on the GPU from the sampler's own coarse-level
    pairs, screens the proposals of levels 4 and 5; the posterior on level 5
    is still the closed-form one, and the logged surrogate error is that of
    the network against the level's linear map."""
    device()
    case("linear-Gaussian closed form, delayed acceptance, 20 seeds")
    s, R, J = 0.15, 20, 2000
    A, E, y = _lin_problem(K=3, nobs=4, s=s, seed=5)
    E = 8.0 * E
    m, C, logZ = _lin_posterior(A + 2.0 ** -10 * E, y, s)
    c = P.Context(2, 5, 3, 1.0, 0.3, 2, s)
    c.set_linear_model(A, E)
    runs = [c.run(to_dev(y), J, J_tilde=100, seed=200 + seed, surrogate=True, sur_collect_max_level=3,
                  sur_da_min_level=4, sur_pairs=8192, sur_epochs=10, sur_hidden=64) for seed in range(R)]
    r0 = runs[0]
    frac = np.mean([r["stage1_passed"] / max(1, r["da_proposed"]) for r in runs])
    print(f"  stage-1 pass fraction {frac:.3f}, surrogate error mean {r0['sur_err_mean']:.3f} "
          f"max {r0['sur_err_max']:.3f} over {r0['sur_err_count']} survivors")
    assert all(r["da_proposed"] > 0 for r in runs)
    assert r0["sur_err_count"] == r0["stage1_passed"]
    da_stages = ~np.isnan(r0["stage_sur_err_mean"])
    assert da_stages.any() and np.all(r0["stage_level"][da_stages] >= 4)
    assert np.all(r0["stage_sur_err_max"][da_stages] >= r0["stage_sur_err_mean"][da_stages])
    _closed_form_check(runs, m, C, logZ, R)
