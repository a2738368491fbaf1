"""GPU checks of the learned surrogate and delayed-acceptance pCN.

* forward and gradients of the BF16-MFMA MLP against the FP64 oracle MLP
  with the same parameters (BF16 operand rounding bounds the difference);
* training on pairs from the GPU's own forward map reduces the loss and
  predicts held-out pairs;
* every delayed-acceptance decision equals the oracle's two-stage rule given
  the same surrogate values and FEM potentials;
* the gain: with the trained surrogate the sampler solves far fewer FEM
  systems per proposal at the delayed-acceptance levels, and its posterior
  agrees with the plain sampler's within Monte Carlo error.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1709_09763_amd as P
from tests import inputs
from tests.gpu_util import case, device, host, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _ctx(K=12, m=3, l_min=3, l_max=5, hidden=64):
    c = P.Context(l_min, l_max, K, 1.0, 0.3, m, 0.01)
    P.mls2mc_surrogate_init(c.h, hidden, 4096, 3)
    return c


def _params(c):
    p = torch.empty(P.mls2mc_surrogate_n_params(c.h), dtype=torch.float32, device="cuda:0")
    P.mls2mc_surrogate_get_params(c.h, p)
    return host(p).astype(np.float64)


def test_surrogate_forward_matches_oracle():
    device()
    case("surrogate forward vs oracle MLP")
    c = _ctx()
    dims = (12, 64, 64, 9)
    x = inputs.theta_batch(1, 300, 12)
    G = torch.empty((300, 9), dtype=torch.float64, device="cuda:0")
    P.mls2mc_surrogate_predict(c.h, to_dev(x), G)
    ref = oracle.mlp_forward(dims, _params(c), x)
    e = rel_err(host(G), ref)
    print(f"  rel err {e:.2e}")
    assert e < 3e-2


def test_surrogate_gradient_matches_oracle():
    device()
    case("surrogate loss/gradient vs oracle MLP")
    c = _ctx()
    dims = (12, 64, 64, 9)
    x = inputs.theta_batch(2, 128, 12)
    t = inputs.theta_batch(3, 128, 9)
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    g = torch.empty(P.mls2mc_surrogate_n_params(c.h), dtype=torch.float32, device="cuda:0")
    P.mls2mc_surrogate_loss_grad(c.h, to_dev(x), to_dev(t), loss, g)
    L_ref, g_ref = oracle.mlp_loss_grad(dims, _params(c), x, t)
    gg = host(g).astype(np.float64)
    e = np.linalg.norm(gg - g_ref) / np.linalg.norm(g_ref)
    print(f"  loss {host(loss)[0]:.6f} vs {L_ref:.6f}, grad rel err {e:.2e}")
    assert abs(host(loss)[0] - L_ref) < 2e-2 * L_ref
    assert e < 3e-2
    # per-layer blocks agree too (no layer silently wrong)
    D, H, O = 12, 64, 9
    cuts = np.cumsum([H * D, H, H * H, H, O * H, O])[:-1]
    for blk, blk_ref in zip(np.split(gg, cuts), np.split(g_ref, cuts)):
        assert np.linalg.norm(blk - blk_ref) <= 5e-2 * np.linalg.norm(blk_ref) + 1e-9


def test_surrogate_training_learns_the_forward_map():
    device()
    case("surrogate training on forward-map pairs")
    K, l = 12, 4
    c = _ctx(K=K, l_min=l, l_max=l, hidden=128)
    P.mls2mc_surrogate_init(c.h, 128, 8192, 5)
    th = to_dev(inputs.theta_batch(4, 8192 + 1024, K, scale=0.7))
    G = c.forward(l, th)
    P.mls2mc_surrogate_add_pairs(c.h, th[:8192].contiguous(), G[:8192].contiguous())
    losses = P.mls2mc_surrogate_train(c.h, 30, 256, 2e-3, 1)
    print(f"  losses {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.1 * losses[0]
    Gp = torch.empty((1024, 9), dtype=torch.float64, device="cuda:0")
    P.mls2mc_surrogate_predict(c.h, th[8192:].contiguous(), Gp)
    Gh, Gt = host(Gp), host(G[8192:])
    e = np.abs(Gh - Gt).mean() / np.abs(Gt - Gt.mean(0)).mean()
    print(f"  held-out error / spread {e:.3f}")
    assert e < 0.2


@pytest.mark.parametrize("mode", ["temper", "bridge"])
def test_delayed_acceptance_decisions_match_oracle_rule(mode):
    device()
    case(f"pcn_step_da {mode}")
    K, m, sn, N = 12, 3, 0.01, 400
    l_lo, l_hi = (4, 4) if mode == "temper" else (4, 5)
    beta, zeta = 0.3, (0.5 if mode == "bridge" else 1.0)
    c = _ctx(K=K, l_min=4, l_max=5)
    # train briefly so the surrogate is informative but imperfect
    th_tr = to_dev(inputs.theta_batch(20, 4096, K))
    P.mls2mc_surrogate_add_pairs(c.h, th_tr, c.forward(4, th_tr))
    P.mls2mc_surrogate_train(c.h, 5, 256, 2e-3, 2)
    th = inputs.theta_batch(21, N, K)
    y = oracle.forward(5, K, 1.0, 0.3, m, inputs.theta_batch(22, 1, K))[0] + sn * inputs.rng(1).standard_normal(9)
    Glo = oracle.forward(l_lo, K, 1.0, 0.3, m, th)
    Ghi = oracle.forward(l_hi, K, 1.0, 0.3, m, th)
    plo = np.array([oracle.potential(g, y, sn) for g in Glo])
    phi = np.array([oracle.potential(g, y, sn) for g in Ghi])
    xi = inputs.theta_batch(23, N, K)
    u1 = 1.0 - inputs.uniforms53(24, N)
    u2 = 1.0 - inputs.uniforms53(25, N)
    thp = oracle.pcn_propose(th, xi, 0.5)
    # the GPU surrogate's values (the oracle judges the rule, not the network)
    Gs = torch.empty((N, 9), dtype=torch.float64, device="cuda:0")
    P.mls2mc_surrogate_predict(c.h, to_dev(th), Gs)
    Gs_old = host(Gs).copy()
    P.mls2mc_surrogate_predict(c.h, to_dev(thp), Gs)
    Gs_new = host(Gs).copy()
    Glp = oracle.forward(l_lo, K, 1.0, 0.3, m, thp)
    Ghp = oracle.forward(l_hi, K, 1.0, 0.3, m, thp)
    plp = np.array([oracle.potential(g, y, sn) for g in Glp])
    php = np.array([oracle.potential(g, y, sn) for g in Ghp])
    acc_ref, s1_ref = [], []
    for j in range(N):
        if mode == "temper":
            po, pn = beta * plo[j], beta * plp[j]
        else:
            po = beta * ((1 - zeta) * plo[j] + zeta * phi[j])
            pn = beta * ((1 - zeta) * plp[j] + zeta * php[j])
        so = beta * oracle.potential(Gs_old[j], y, sn)
        snw = beta * oracle.potential(Gs_new[j], y, sn)
        a, s1 = oracle.da_accept(po, pn, so, snw, u1[j], u2[j])
        acc_ref.append(a)
        s1_ref.append(s1)
    acc_ref, s1_ref = np.array(acc_ref), np.array(s1_ref)
    T, GL, GH, PL, PH = to_dev(th), to_dev(Glo), to_dev(Ghi), to_dev(plo), to_dev(phi)
    acc = torch.empty(N, dtype=torch.uint8, device="cuda:0")
    s1 = torch.empty(N, dtype=torch.uint8, device="cuda:0")
    nlo = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    nhi = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    P.mls2mc_pcn_step_da(c.h, l_lo, l_hi, beta, zeta, 0.5, T, GL, GH if mode == "bridge" else None, PL,
                         PH if mode == "bridge" else None, to_dev(y), to_dev(xi), to_dev(u1), to_dev(u2),
                         acc, s1, nlo, nhi)
    np.testing.assert_array_equal(host(s1).astype(bool), s1_ref)
    np.testing.assert_array_equal(host(acc).astype(bool), acc_ref)
    assert 0 < s1_ref.sum() < N and 0 < acc_ref.sum()
    assert host(nlo)[0] == s1_ref.sum()
    if mode == "bridge":
        assert host(nhi)[0] == s1_ref.sum()
    th_ref = np.where(acc_ref[:, None], thp, th)
    assert rel_err(host(T), th_ref) < 1e-15
    assert rel_err(host(GL), np.where(acc_ref[:, None], Glp, Glo)) < 1e-10


def _moves_at(r, J, n_mcmc, lmin):
    """accepted pCN moves on the stages whose level is >= lmin"""
    sel = r["stage_level"] >= lmin
    return float(np.sum(r["stage_acc_rate"][sel]) * J * n_mcmc)


def _rel_err_paper(mean, ref, lam):
    """the paper's relative error of a posterior mean, Lambda^{1/2}-weighted l1 (Sec. 5.1)"""
    w = np.sqrt(lam)
    return float(np.abs(w * (mean - ref)).sum() / np.abs(w * ref).sum())


def test_surrogate_gain_in_the_sampler():
    """What the trained network gains on the delayed-acceptance levels
    (h = 1/32, 1/64): the chain still moves (accepted moves comparable to
    the plain sampler's) while far fewer proposals reach the FEM solve, so
    accepted moves per FEM solve improve; and the posterior mean is as
    accurate (the paper's relative error against the mean pooled over four
    seeds of each form)."""
    device()
    case("sampler with vs without surrogate, 4 seeds")
    K, m, sn, J, n_mcmc = 20, 5, 0.005, 1000, 5
    c = P.Context(3, 6, K, 1.0, 0.3, m, sn)
    lam = c.kl_eigenvalues()
    th_true = inputs.theta_batch(30, 1, K)
    y = to_dev(oracle.forward(6, K, 1.0, 0.3, m, th_true)[0] + sn * inputs.rng(31).standard_normal(m * m))
    plain, da = [], []
    for seed in (4, 5, 6, 7):
        plain.append(c.run(y, J, seed=seed))
        da.append(c.run(y, J, seed=seed, surrogate=True, sur_collect_max_level=4, sur_da_min_level=5,
                        sur_pairs=20480, sur_epochs=30, sur_hidden=128))
    for p_, d_ in zip(plain, da):
        frac = d_["stage1_passed"] / max(1, d_["da_proposed"])
        mp, md = _moves_at(p_, J, n_mcmc, 5), _moves_at(d_, J, n_mcmc, 5)
        sp, sd_ = sum(p_["solves"][5:7]), sum(d_["solves"][5:7])
        print(f"  plain {p_['seconds']:.2f}s: {mp:.0f} moves / {sp} solves on h <= 1/32; "
              f"DA {d_['seconds']:.2f}s: {md:.0f} moves / {sd_} solves, stage-1 pass {frac:.3f}, "
              f"surrogate error {d_['sur_err_mean']:.2f} (max {d_['sur_err_max']:.2f}) sigma_n")
        assert d_["da_proposed"] > 0
        assert frac < 0.6  # most proposals never reach the FEM solve
        assert sd_ < 0.7 * sp
        assert md > 0.5 * mp  # the chain does not stall behind the screen
        assert md / sd_ > 1.1 * (mp / sp)  # more accepted moves per FEM solve
        assert d_["sur_err_count"] == d_["stage1_passed"] and d_["sur_err_mean"] > 0
    pooled = np.mean([host(r["theta"]).mean(0) for r in plain + da], axis=0)
    e_plain = np.mean([_rel_err_paper(host(r["theta"]).mean(0), pooled, lam) for r in plain])
    e_da = np.mean([_rel_err_paper(host(r["theta"]).mean(0), pooled, lam) for r in da])
    print(f"  RelErr vs the pooled mean: plain {e_plain:.3f}, DA {e_da:.3f}")
    assert e_da < 1.5 * e_plain + 0.02


def test_delayed_acceptance_across_forward_chunks():
    """At h = 1/512 the second-stage solves of the screened proposals run in
    2 GiB chunks of 512 with a device-side count.  With about 650 of 700
    proposals passing the first stage, the count crosses a chunk boundary;
    every decision must still follow the two-stage rule applied to the plain
    forward map's potentials, and the accepted particles must carry the plain
    forward map's observations."""
    device()
    K, m, sn, N, l, beta = 12, 3, 0.1, 700, 9, 0.3
    case(f"pcn_step_da chunks l={l} N={N}")
    c = P.Context(l, l, K, 1.0, 0.3, m, sn)
    P.mls2mc_surrogate_init(c.h, 64, 4096, 3)
    th = inputs.theta_batch(31, N, K)
    xi = inputs.theta_batch(32, N, K)
    thp = oracle.pcn_propose(th, xi, 0.5)
    y = host(c.forward(l, to_dev(inputs.theta_batch(33, 1, K))))[0] + sn * inputs.rng(3).standard_normal(9)
    Glo, Glp = host(c.forward(l, to_dev(th))), host(c.forward(l, to_dev(thp)))
    plo = np.array([oracle.potential(g, y, sn) for g in Glo])
    plp = np.array([oracle.potential(g, y, sn) for g in Glp])
    u1 = 1.0 - inputs.uniforms53(34, N)
    u1[:650] = 1e-300  # the first stage passes these unless the surrogate's
    # potential rises by more than 690 (sigma = 0.1 keeps it well below that)
    u2 = 1.0 - inputs.uniforms53(35, N)
    Gs = torch.empty((N, 9), dtype=torch.float64, device="cuda:0")
    P.mls2mc_surrogate_predict(c.h, to_dev(th), Gs)
    Gs_old = host(Gs).copy()
    P.mls2mc_surrogate_predict(c.h, to_dev(thp), Gs)
    Gs_new = host(Gs).copy()
    ref = [oracle.da_accept(beta * plo[j], beta * plp[j], beta * oracle.potential(Gs_old[j], y, sn),
                            beta * oracle.potential(Gs_new[j], y, sn), u1[j], u2[j]) for j in range(N)]
    acc_ref = np.array([a for a, _ in ref])
    s1_ref = np.array([s for _, s in ref])
    print(f"  stage 1 passed {s1_ref.sum()}, accepted {acc_ref.sum()} of {N}")
    assert s1_ref.sum() > 512 and 0 < acc_ref.sum() < N
    T, GL, PL = to_dev(th), to_dev(Glo), to_dev(plo)
    acc = torch.empty(N, dtype=torch.uint8, device="cuda:0")
    s1 = torch.empty(N, dtype=torch.uint8, device="cuda:0")
    nlo = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    P.mls2mc_pcn_step_da(c.h, l, l, beta, 1.0, 0.5, T, GL, None, PL, None, to_dev(y), to_dev(xi),
                         to_dev(u1), to_dev(u2), acc, s1, nlo, None)
    np.testing.assert_array_equal(host(s1).astype(bool), s1_ref)
    np.testing.assert_array_equal(host(acc).astype(bool), acc_ref)
    assert host(nlo)[0] == s1_ref.sum()
    # proposals are formed on the device, so the solved inputs may differ from
    # the host's in the last bit: the kept observations are the plain forward
    # map's to the solver's tolerance, the rejected ones untouched
    GLh = host(GL)
    np.testing.assert_array_equal(GLh[~acc_ref], Glo[~acc_ref])
    assert rel_err(GLh[acc_ref], Glp[acc_ref]) < 1e-10
    assert rel_err(host(T), np.where(acc_ref[:, None], thp, th)) < 1e-15


# ---- the network of the configured surrogate: 100 -> 256 -> 256 -> 49 ----
# Element-by-element tolerances from the arithmetic.  Every matrix product
# of the library rounds both operands to BF16 (round to nearest: a relative
# error of up to u = 2^-8, spread evenly) and sums in FP32; the bias
# gradients are FP32 row sums.  To first order each output or gradient
# entry then errs by a linear combination of the independent rounding errors
# of all operands, with correlations the network's structure fixes (one
# rounded weight serves the whole batch, one rounded activation every unit
# of the next layer).  Its standard deviation is estimated by propagating
# independent random relative perturbations, uniform in [-u, u], through
# the same products (TRIALS times, in FP64); every error must lie within
# NSIG of it.  The reference values themselves are the oracle's.
U = 2.0 ** -8
NSIG = 8.0
TRIALS = 32
BIG = (100, 256, 256, 49)


def _split(p, dims):
    D, H1, H2, O = dims
    sizes = [H1 * D, H1, H2 * H1, H2, O * H2, O]
    W1, b1, W2, b2, W3, b3 = np.split(p, np.cumsum(sizes)[:-1])
    return W1.reshape(H1, D), b1, W2.reshape(H2, H1), b2, W3.reshape(O, H2), b3


def _gelu(z):
    from scipy.special import erf
    cdf = 0.5 * (1.0 + erf(z / np.sqrt(2.0)))
    return z * cdf, cdf + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _net(p, x, t, rnd):
    """outputs and gradients with every BF16 operand passed through rnd"""
    W1, b1, W2, b2, W3, b3 = _split(p, BIG)
    z1 = rnd(x) @ rnd(W1).T + b1
    h1, d1 = _gelu(z1)
    z2 = rnd(h1) @ rnd(W2).T + b2
    h2, d2 = _gelu(z2)
    out = rnd(h2) @ rnd(W3).T + b3
    if t is None:
        return out, None
    g3 = (out - t) / t.size
    g2 = (rnd(g3) @ rnd(W3)) * d2
    g1 = (rnd(g2) @ rnd(W2)) * d1
    grad = [rnd(g1).T @ rnd(x), g1.sum(0), rnd(g2).T @ rnd(h1), g2.sum(0), rnd(g3).T @ rnd(h2), g3.sum(0)]
    return out, np.concatenate([v.ravel() for v in grad])


def _rounding_sd(p, x, t=None, seed=0):
    g = np.random.default_rng(seed)
    o0, d0 = _net(p, x, t, lambda a: a)
    so, sg = np.zeros_like(o0), (None if d0 is None else np.zeros_like(d0))
    for _ in range(TRIALS):
        o, d = _net(p, x, t, lambda a: a * (1.0 + U * g.uniform(-1.0, 1.0, a.shape)))
        so += (o - o0) ** 2
        if d is not None:
            sg += (d - d0) ** 2
    return np.sqrt(so / TRIALS), (None if d0 is None else np.sqrt(sg / TRIALS))


def test_configured_surrogate_forward_elementwise():
    device()
    case("surrogate 100-256-256-49 forward, element by element")
    c = P.Context(3, 4, 100, 1.0, 0.3, 7, 0.002)
    P.mls2mc_surrogate_init(c.h, 256, 4096, 11)
    assert P.mls2mc_surrogate_n_params(c.h) == 100 * 256 + 256 + 256 * 256 + 256 + 49 * 256 + 49
    x = inputs.theta_batch(40, 1000, 100)
    G = torch.empty((1000, 49), dtype=torch.float64, device="cuda:0")
    P.mls2mc_surrogate_predict(c.h, to_dev(x), G)
    p = _params(c)
    ref = oracle.mlp_forward(BIG, p, x)
    sd, _ = _rounding_sd(p, x)
    bound = NSIG * sd + 1e-7 * np.abs(ref).max()
    err = np.abs(host(G) - ref)
    print(f"  max err / bound {np.max(err / bound):.3f}, max rel err {rel_err(host(G), ref):.2e}")
    assert np.all(err <= bound)


def test_configured_surrogate_gradient_elementwise():
    """per-parameter gradients of the 100-256-256-49 network at batch 512
    (two 128-wide k rounds in the hidden-layer products) against the oracle"""
    device()
    case("surrogate 100-256-256-49 gradient, element by element")
    B = 512
    c = P.Context(3, 4, 100, 1.0, 0.3, 7, 0.002)
    P.mls2mc_surrogate_init(c.h, 256, 4096, 12)
    x = inputs.theta_batch(41, B, 100)
    t = inputs.theta_batch(42, B, 49)
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    g = torch.empty(P.mls2mc_surrogate_n_params(c.h), dtype=torch.float32, device="cuda:0")
    P.mls2mc_surrogate_loss_grad(c.h, to_dev(x), to_dev(t), loss, g)
    p = _params(c)
    L_ref, g_ref = oracle.mlp_loss_grad(BIG, p, x, t)
    sd_out, sd = _rounding_sd(p, x, t, seed=1)
    gg = host(g).astype(np.float64)
    err = np.abs(gg - g_ref)
    D, H, O = 100, 256, 49
    cuts = np.cumsum([H * D, H, H * H, H, O * H, O])[:-1]
    ok = True
    for nm, e, v, gr in zip(["W1", "b1", "W2", "b2", "W3", "b3"], np.split(err, cuts), np.split(sd, cuts),
                            np.split(g_ref, cuts)):
        bound = NSIG * v + 1e-6 * np.abs(gr).max()
        print(f"  {nm}: max err / bound {np.max(e / bound):.3f}, max rel err {e.max() / np.abs(gr).max():.2e}")
        ok &= bool(np.all(e <= bound))
    # the loss, half the mean square of the outputs' errors
    out = oracle.mlp_forward(BIG, p, x)
    sd_L = np.sqrt(np.sum(((out - t) * sd_out) ** 2)) / t.size
    print(f"  loss {host(loss)[0]:.6f} vs {L_ref:.6f} (sd {sd_L:.2e})")
    assert ok
    assert abs(host(loss)[0] - L_ref) <= NSIG * sd_L + 1e-6 * L_ref
