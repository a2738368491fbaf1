"""Pins of the oracle's MLS^2MC sampler (Sec. 4) against closed forms.

* Linear-Gaussian model G_l(theta) = (A + 2^{-2l} E) theta with a N(0, I)
  prior: the posterior on the finest level is Gaussian with covariance
  (I + A^T A / s^2)^{-1} and the evidence has a closed form (Sec. 2.1).
* The number of forward evaluations per level follows the cost model of
  Prop. 4.4, adapted to n pCN steps per stage and the J_tilde look-ahead
  evaluations of Sec. 4.4.
* With l_min = l_max the sampler is single-level SMC (Example 4.1).
* A PDE model with K = 1 has a posterior computable by quadrature.
"""
import numpy as np
import pytest

import oracle
from tests import inputs


def _lin_problem(K=3, nobs=4, s=0.2, seed=0):
    g = inputs.rng(seed)
    A = g.standard_normal((nobs, K))
    E = g.standard_normal((nobs, K))
    th = g.standard_normal(K)
    y = A @ th + s * g.standard_normal(nobs)
    return A, E, y


def _lin_posterior(A, y, s):
    K = A.shape[1]
    P = np.eye(K) + A.T @ A / s ** 2
    C = np.linalg.inv(P)
    m = C @ A.T @ y / s ** 2
    G = s ** 2 * np.eye(len(y)) + A @ A.T
    logZ = -0.5 * np.linalg.slogdet(P)[1] - 0.5 * y @ np.linalg.solve(G, y)
    return m, C, logZ


def _expected_solves(r, J, Jt, n_mcmc, l_min):
    ex = np.zeros(16, dtype=np.int64)
    ex[l_min] += J
    for typ, lev, z in zip(r["stage_type"], r["stage_level"], r["stage_zeta"]):
        if typ in (0, 1):
            ex[lev] += n_mcmc * J
            if typ == 1:
                ex[lev + 1] += Jt
        else:
            if typ in (2, 3):
                ex[lev] += J  # first evaluation of all particles on the finer level
            ex[lev] += n_mcmc * J
            if z < 1.0:
                ex[lev - 1] += n_mcmc * J
    return ex


@pytest.mark.slow
@pytest.mark.parametrize("s_adapt,kernel", [(False, 0), (True, 0), (False, 1)])
def test_linear_gaussian_single_level_posterior_and_evidence(s_adapt, kernel):
    # the optional step adaptation changes the step only between stages, so
    # every mutation kernel still leaves its tempered target invariant; the
    # random-walk kernel (kernel 1) needs the prior ratio in its acceptance
    s = 0.2
    A, E, y = _lin_problem(s=s)
    m, C, logZ = _lin_posterior(A + 2.0 ** -6 * E, y, s)
    R, J = 8, 2000
    means, vars_, lz = [], [], []
    step = 2.38 / np.sqrt(3) if kernel == 1 else 0.5
    for seed in range(R):
        r = oracle.run_sampler(y, model="linear", l_min=3, l_max=3, K=3, nobs=4, sigma_n=s, J=J,
                               seed=seed, lin_A=A, lin_E=E, n_mcmc=5, s_adapt=s_adapt, kernel=kernel,
                               s_pcn=step)
        assert np.all(r["stage_type"] == 0)  # single-level SMC
        means.append(r["theta"].mean(0))
        vars_.append(r["theta"].var(0))
        lz.append(r["log_Z"])
    means, vars_, lz = map(np.array, (means, vars_, lz))
    se = means.std(0, ddof=1) / np.sqrt(R)
    assert np.all(np.abs(means.mean(0) - m) < 4 * se + 0.02 * np.sqrt(np.diag(C))), (means.mean(0), m)
    np.testing.assert_allclose(vars_.mean(0), np.diag(C), rtol=0.1)
    assert abs(lz.mean() - logZ) < 4 * lz.std(ddof=1) / np.sqrt(R) + 0.05, (lz.mean(), logZ)


@pytest.mark.slow
@pytest.mark.parametrize("scheme,dep", [(0, 30.0), (1, 3.0)])
def test_linear_gaussian_multilevel_posterior(scheme, dep):
    # scheme 0: the adaptive MLS^2MC scheme, with strong level dependence
    # (coarse levels are poor models); scheme 1: multilevel bridging, with
    # moderate dependence (with strong dependence its evidence estimate is
    # heavy-tailed, see test_mlb_evidence_spread)
    s = 0.15
    A, E, y = _lin_problem(K=2, nobs=3, s=s, seed=3)
    E = dep * E
    m, C, logZ = _lin_posterior(A + 2.0 ** -10 * E, y, s)
    R, J = 8, 2000
    means, lz = [], []
    kinds = set()
    for seed in range(R):
        r = oracle.run_sampler(y, model="linear", l_min=2, l_max=5, K=2, nobs=3, sigma_n=s, J=J,
                               J_tilde=100, seed=100 + seed, lin_A=A, lin_E=E, scheme=scheme)
        assert r["final_level"] == 5 and r["final_beta"] == 1.0
        kinds |= set(r["stage_type"].tolist())
        means.append(r["theta"].mean(0))
        lz.append(r["log_Z"])
        ex = _expected_solves(r, J, 100, 5, 2)
        np.testing.assert_array_equal(np.array(r["solves"]), ex)
    # bridging path (posterior at level 5 is A + 2^-10 E)
    means, lz = np.array(means), np.array(lz)
    se = means.std(0, ddof=1) / np.sqrt(R)
    assert np.all(np.abs(means.mean(0) - m) < 4 * se + 0.03 * np.sqrt(np.diag(C))), (means.mean(0), m)
    assert abs(lz.mean() - logZ) < 4 * lz.std(ddof=1) / np.sqrt(R) + 0.1
    assert 0 in kinds and (2 in kinds or 3 in kinds)
    if scheme == 1:
        assert kinds <= {0, 3, 4}  # no look-ahead in multilevel bridging


def test_first_update_is_tempering_and_levels_monotone():
    s = 0.3
    A, E, y = _lin_problem(seed=5)
    r = oracle.run_sampler(y, model="linear", l_min=1, l_max=4, K=3, nobs=4, sigma_n=s, J=300,
                           J_tilde=50, seed=1, lin_A=A, lin_E=10 * E)
    assert r["stage_type"][0] == 0 and r["stage_level"][0] == 1
    assert np.all(np.diff(r["stage_level"]) >= 0)
    b = r["stage_beta"]
    assert np.all(np.diff(b) >= 0) and b[-1] == 1.0
    # every tempering update right after a level update is taken without a look-ahead
    t = r["stage_type"]
    for i in range(1, len(t)):
        if t[i] in (0, 1) and t[i - 1] in (2, 3, 4):
            assert t[i] == 0
    np.testing.assert_array_equal(np.array(r["solves"]), _expected_solves(r, 300, 50, 5, 1))


@pytest.mark.slow
def test_mlb_evidence_spread():
    # When the coarse levels are poor models, bridging at beta = 1 (MLB)
    # spreads the log-evidence estimate far more than MLS^2MC, which bridges
    # at the smaller temperatures its look-ahead picks (the paper's Sec. 5
    # comparison); both stay consistent where the levels agree better.
    s = 0.15
    A, E, y = _lin_problem(K=2, nobs=3, s=s, seed=3)
    spread = {}
    for scheme in (0, 1):
        lz = [oracle.run_sampler(y, model="linear", l_min=2, l_max=5, K=2, nobs=3, sigma_n=s, J=2000,
                                 J_tilde=100, seed=100 + sd, lin_A=A, lin_E=30.0 * E, scheme=scheme)["log_Z"]
              for sd in range(16)]
        spread[scheme] = np.std(lz, ddof=1)
    assert spread[1] > 4 * spread[0], spread


def test_mlb_scheme_path_and_solves():
    # multilevel bridging: temper on l_min up to beta = 1, then bridge level
    # by level at beta = 1 (no look-ahead solves)
    A, E, y = _lin_problem(seed=8)
    J, Jt = 300, 50
    r = oracle.run_sampler(y, model="linear", l_min=1, l_max=4, K=3, nobs=4, sigma_n=0.3, J=J, J_tilde=Jt,
                           seed=2, lin_A=A, lin_E=10 * E, scheme=1)
    t, lv, b = r["stage_type"], r["stage_level"], r["stage_beta"]
    k = int(np.argmax(b == 1.0))
    assert np.all(t[:k + 1] == 0) and np.all(lv[:k + 1] == 1)
    assert np.all(np.isin(t[k + 1:], (3, 4))) and np.all(b[k:] == 1.0)
    assert r["final_level"] == 4 and r["final_beta"] == 1.0
    np.testing.assert_array_equal(np.array(r["solves"]), _expected_solves(r, J, Jt, 5, 1))


def test_adaptive_max_level():
    # scheme u' (tau_min > 0): at beta = 1 the run stops once a level update
    # would change the measure by cv^LU < tau_min
    A, E, y = _lin_problem(seed=9)
    J, Jt = 300, 50
    kw = dict(model="linear", l_min=1, l_max=4, K=3, nobs=4, sigma_n=0.3, J=J, J_tilde=Jt, seed=3, lin_A=A)
    # identical levels: cv^LU = 0, so u tempers on l_min and u' stops there
    r0 = oracle.run_sampler(y, lin_E=0 * E, **kw)
    r1 = oracle.run_sampler(y, lin_E=0 * E, tau_min=1e-3, **kw)
    assert r0["final_level"] == 4 and r1["final_level"] == 1 and r1["final_beta"] == 1.0
    ex = _expected_solves(r1, J, Jt, 5, 1)
    ex[2] += Jt  # the look-ahead that decided to stop
    np.testing.assert_array_equal(np.array(r1["solves"]), ex)
    # strongly different levels and a tiny tau_min: the same path as u, with
    # the level updates at beta = 1 opened by a look-ahead
    r0 = oracle.run_sampler(y, lin_E=20 * E, **kw)
    r1 = oracle.run_sampler(y, lin_E=20 * E, tau_min=1e-12, **kw)
    assert r0["final_level"] == r1["final_level"] == 4
    np.testing.assert_array_equal(r0["stage_level"], r1["stage_level"])
    np.testing.assert_array_equal(r0["stage_beta"], r1["stage_beta"])
    np.testing.assert_array_equal(r0["theta"], r1["theta"])
    forced = (r0["stage_type"] == 3)
    np.testing.assert_array_equal(r1["stage_type"][forced], 2)
    np.testing.assert_array_equal(np.array(r1["solves"]), _expected_solves(r1, J, Jt, 5, 1))


def test_random_walk_proposal():
    th = inputs.rng(5).standard_normal((4, 3))
    xi = inputs.rng(6).standard_normal((4, 3))
    np.testing.assert_array_equal(oracle.rwm_propose(0.7, th, xi), th + 0.7 * xi)


def test_step_adaptation_schedule():
    A, E, y = _lin_problem(seed=7)
    kw = dict(model="linear", l_min=1, l_max=3, K=3, nobs=4, sigma_n=0.05, J=300, J_tilde=50,
              seed=4, lin_A=A, lin_E=5 * E, s_pcn=0.9)
    fixed = oracle.run_sampler(y, **kw)
    np.testing.assert_array_equal(fixed["stage_step"], 0.9)
    r = oracle.run_sampler(y, s_adapt=True, **kw)
    st, a = r["stage_step"], r["stage_acc_rate"]
    assert st[0] == 0.9 and len(st) > 3
    # each stage's step follows from the previous stage's step and acceptance
    # rate: it grows iff that rate exceeded 1/4, and stays in [0.005, 1]
    for k in range(1, len(st)):
        want = min(1.0, max(0.005, st[k - 1] * np.exp(2.0 * (a[k - 1] - 0.25))))
        assert abs(st[k] - want) <= 1e-15 * want
        assert (st[k] > st[k - 1]) == (a[k - 1] > 0.25) or st[k] in (0.005, 1.0)
    # small noise: the fixed step's acceptance collapses, the adapted one stays nearer 1/4
    assert abs(np.mean(a[-3:]) - 0.25) < abs(np.mean(fixed["stage_acc_rate"][-3:]) - 0.25)


def test_deterministic_replay():
    A, E, y = _lin_problem(seed=6)
    kw = dict(model="linear", l_min=1, l_max=3, K=3, nobs=4, sigma_n=0.3, J=200, J_tilde=40,
              seed=9, lin_A=A, lin_E=E)
    r1 = oracle.run_sampler(y, **kw)
    r2 = oracle.run_sampler(y, **kw)
    np.testing.assert_array_equal(r1["theta"], r2["theta"])
    assert r1["log_Z"] == r2["log_Z"]


@pytest.mark.slow
def test_pde_brute_force_posterior_k1():
    # K = 1 on the real PDE at h = 1/8: posterior mean and variance by
    # quadrature on a fine grid against the SMC estimate
    l, K, m, sn = 3, 1, 3, 0.02
    th_true = np.array([[0.8]])
    y = oracle.forward(l, K, 1.0, 0.3, m, th_true)[0] + sn * inputs.rng(0).standard_normal(m * m)
    grid = np.linspace(-6, 6, 4001)
    G = oracle.forward(l, K, 1.0, 0.3, m, grid[:, None])
    phi = 0.5 * (((G - y) / sn) ** 2).sum(1)
    lp = -phi - 0.5 * grid ** 2
    wq = np.exp(lp - lp.max())
    wq /= wq.sum()
    mq = (wq * grid).sum()
    vq = (wq * (grid - mq) ** 2).sum()
    R, J = 6, 1500
    ms, vs = [], []
    for seed in range(R):
        r = oracle.run_sampler(y, l_min=l, l_max=l, K=K, m=m, sigma_n=sn, J=J, seed=seed)
        ms.append(r["theta"].mean())
        vs.append(r["theta"].var())
    ms = np.array(ms)
    se = ms.std(ddof=1) / np.sqrt(R)
    assert abs(ms.mean() - mq) < 4 * se + 0.02 * np.sqrt(vq), (ms.mean(), mq, se)
    assert abs(np.mean(vs) / vq - 1) < 0.15, (np.mean(vs), vq)


def test_delayed_acceptance_rule_special_cases():
    rng = inputs.rng(77)
    for _ in range(2000):
        po, pn = rng.normal(0, 3, 2)
        u1, u2 = 1.0 - inputs.uniforms53(int(rng.integers(1 << 30)), 2)
        # perfect surrogate: stage 2 always accepts after stage 1
        a, s1 = oracle.da_accept(po, pn, po, pn, u1, u2)
        assert a == s1
        # constant surrogate: stage 1 always passes; stage 2 is plain MH with u2
        a, s1 = oracle.da_accept(po, pn, 5.0, 5.0, u1, u2)
        assert s1 and a == oracle.mh_accept(po, pn, u2)
    # stage 1 rejects -> no move, whatever stage 2 would say
    a, s1 = oracle.da_accept(0.0, -100.0, 0.0, 100.0, 0.5, 0.5)
    assert not s1 and not a


@pytest.mark.slow
def test_delayed_acceptance_keeps_linear_gaussian_posterior():
    # a deliberately poor surrogate (perturbed forward matrix) must not bias
    # the posterior: the two-stage rule is exact for any surrogate
    s = 0.2
    A, E, y = _lin_problem(s=s, seed=11)
    m, C, logZ = _lin_posterior(A + 2.0 ** -6 * E, y, s)
    S = A + 0.3 * inputs.rng(12).standard_normal(A.shape)
    R, J = 8, 2000
    means, vars_, pass_frac = [], [], []
    for seed in range(R):
        r = oracle.run_sampler(y, model="linear", l_min=3, l_max=3, K=3, nobs=4, sigma_n=s, J=J,
                               seed=300 + seed, lin_A=A, lin_E=E, da_S=S)
        means.append(r["theta"].mean(0))
        vars_.append(r["theta"].var(0))
        pass_frac.append(r["stage1_passed"] / r["proposed"])
    means = np.array(means)
    se = means.std(0, ddof=1) / np.sqrt(R)
    assert np.all(np.abs(means.mean(0) - m) < 4 * se + 0.02 * np.sqrt(np.diag(C)))
    np.testing.assert_allclose(np.mean(vars_, 0), np.diag(C), rtol=0.1)
    assert 0.05 < np.mean(pass_frac) < 0.95  # the surrogate does filter


@pytest.mark.slow
def test_flowcell_brute_force_posterior_k1():
    # the flow-cell model (Example 5.3) with K = 1 at h = 1/8: posterior mean
    # and variance by quadrature against the SMC estimate of the sampler run
    # on that model
    l, K, m, sn = 3, 1, 3, 0.01
    B = oracle.kl_basis(l, K, 1.0, 0.3)

    def G_of(th):
        return oracle.flow_forward_kappa(l, m, np.exp(oracle.kl_field(l, B, th[:, None])))

    y = G_of(np.array([0.9]))[0] + sn * inputs.rng(1).standard_normal(m * m)
    grid = np.linspace(-6, 6, 4001)
    phi = 0.5 * (((G_of(grid) - y) / sn) ** 2).sum(1)
    lp = -phi - 0.5 * grid ** 2
    wq = np.exp(lp - lp.max())
    wq /= wq.sum()
    mq = (wq * grid).sum()
    vq = (wq * (grid - mq) ** 2).sum()
    R, J = 6, 1500
    ms, vs = [], []
    for seed in range(R):
        r = oracle.run_sampler(y, model="flowcell", l_min=l, l_max=l, K=K, m=m, sigma_n=sn, J=J, seed=seed)
        ms.append(r["theta"].mean())
        vs.append(r["theta"].var())
    ms = np.array(ms)
    se = ms.std(ddof=1) / np.sqrt(R)
    assert abs(ms.mean() - mq) < 4 * se + 0.02 * np.sqrt(vq), (ms.mean(), mq, se)
    assert abs(np.mean(vs) / vq - 1) < 0.15, (np.mean(vs), vq)


def test_stored_oracle_runs_are_the_oracles():
    """tests/golden/oracle_runs.json holds what its generator's cases give:
    the same cases, and for the cheapest one the same result as a fresh
    oracle run, value for value."""
    import json
    import os
    from tests.golden import make_oracle_runs as mk
    rec = json.load(open(mk.OUT))
    assert set(rec) == set(mk.CASES)
    for name, c in mk.CASES.items():
        assert rec[name]["case"] == json.loads(json.dumps(c))
    fresh = json.loads(json.dumps(mk.run_case(mk.CASES["batch_J384_l6_s0"])))
    assert fresh == rec["batch_J384_l6_s0"]["result"]
    assert os.path.basename(mk.OUT) == "oracle_runs.json"
