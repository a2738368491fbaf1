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


def test_surrogate_gain_in_the_sampler():
    """the trained network screens proposals: far fewer FEM solves per
    proposal on the delayed-acceptance levels, same posterior (MC error)"""
    device()
    case("sampler with vs without surrogate")
    K, m, sn, J = 20, 5, 0.005, 1000
    c = P.Context(3, 6, K, 1.0, 0.3, m, sn)
    th_true = inputs.theta_batch(30, 1, K)
    y = to_dev(oracle.forward(6, K, 1.0, 0.3, m, th_true)[0] + sn * inputs.rng(31).standard_normal(m * m))
    plain = c.run(y, J, seed=4)
    da = c.run(y, J, seed=4, surrogate=True, sur_collect_max_level=4, sur_da_min_level=5, sur_pairs=20480,
               sur_epochs=30, sur_hidden=128)
    frac = da["stage1_passed"] / max(1, da["da_proposed"])
    acc_plain = plain["accepted"] / plain["proposed"]
    print(f"  plain: {plain['seconds']:.2f}s solves {plain['solves'][3:7]} acc {acc_plain:.3f}")
    print(f"  DA:    {da['seconds']:.2f}s solves {da['solves'][3:7]} stage-1 pass {frac:.3f} "
          f"train {da['sur_train_seconds']:.2f}s loss {da['sur_final_loss']:.4f}")
    assert da["da_proposed"] > 0
    assert frac < 0.6  # most proposals never reach the FEM solve
    assert sum(da["solves"][5:7]) < 0.7 * sum(plain["solves"][5:7])
    a = host(plain["theta"])
    b = host(da["theta"])
    sd = np.sqrt(0.5 * (a.var(0) + b.var(0)))
    # pCN particles are correlated: allow an effective sample size of J/10
    assert np.all(np.abs(a.mean(0) - b.mean(0)) < 5 * sd * np.sqrt(2 / (J / 10)))


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
