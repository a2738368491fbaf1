"""GPU parity of the forward map (Sec. 5 model; Sec. 2.1 forward response):
KL field GEMM, multigrid-PCG solve and observation, against the CPU oracle
(banded Cholesky) on the same inputs.  FP64 bar: rel 1e-10 on G and p."""
import numpy as np
import pytest
import torch

import oracle
import paper_1709_09763_amd as P
from tests import inputs
from tests.gpu_util import case, device, host, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("l", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("K", [10, 50])
def test_kl_field_parity(l, K):
    device()
    case(f"kl_field l={l} K={K}")
    ctx = P.Context(l, l, K, 1.0, 0.3, 3, 0.01)
    th = inputs.theta_batch(l * 10 + K, 67, K)
    a = host(ctx.kl_field(l, to_dev(th), P.FIELD_LOG_F64))
    B = oracle.kl_basis(l, K, 1.0, 0.3)
    ref = th @ B
    assert rel_err(a, ref) < 1e-12
    kap = host(ctx.kl_field(l, to_dev(th), P.FIELD_KAPPA_F64))
    assert np.abs(kap / np.exp(ref) - 1).max() < 1e-12


@pytest.mark.parametrize("corr", [0.3, 0.1])
def test_kl_basis_large_K(corr):
    device()
    l, K = 4, 200
    case(f"kl_field l={l} K={K} corr={corr}")
    ctx = P.Context(l, l, K, 1.0, corr, 3, 0.01)
    eye = np.eye(K)
    Bg = host(ctx.kl_field(l, to_dev(eye), P.FIELD_LOG_F64))
    Bo = oracle.kl_basis(l, K, 1.0, corr)
    assert rel_err(Bg, Bo) < 1e-12


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5, 6, 7])
def test_forward_field_parity(l):
    device()
    N = 37  # ragged against every grid shape
    case(f"forward_field l={l} N={N}")
    m = 5
    ctx = P.Context(l, l, 4, 1.0, 0.3, m, 0.01)
    kap = inputs.kappa_batch(100 + l, N, oracle.n_elem(l), spread=1.0)
    G, p, st, it = ctx.forward_field(l, to_dev(kap), want_p=True)
    Gr, pr = oracle.forward_kappa(l, m, kap, want_p=True)
    assert (host(st) == 0).all()
    assert rel_err(host(G), Gr) < 1e-10
    assert rel_err(host(p), pr) < 1e-10
    print(f"  iters min/mean/max {host(it).min()}/{host(it).mean():.1f}/{host(it).max()}")


@pytest.mark.parametrize("cfg", [
    dict(name="single-level h=1/16", levels=[4], K=10, m=3, N=200),
    dict(name="multilevel h=1/8..1/64", levels=[3, 4, 5, 6], K=50, m=5, N=96),
])
def test_forward_parity_workloads(cfg):
    device()
    ctx = P.Context(min(cfg["levels"]), max(cfg["levels"]), cfg["K"], 1.0, 0.3, cfg["m"], 0.01)
    th = inputs.theta_batch(7, cfg["N"], cfg["K"])
    for l in cfg["levels"]:
        case(f"forward {cfg['name']} l={l}")
        G, st, it = ctx.forward(l, to_dev(th), with_stats=True)
        Gr = oracle.forward(l, cfg["K"], 1.0, 0.3, cfg["m"], th)
        assert (host(st) == 0).all()
        assert rel_err(host(G), Gr) < 1e-10


def test_forward_strong_contrast():
    device()
    l, N = 6, 16
    case(f"forward_field contrast l={l}")
    ctx = P.Context(l, l, 4, 1.0, 0.3, 7, 0.01)
    kap = inputs.kappa_batch(5, N, oracle.n_elem(l), spread=2.5)  # e^{+-7} per element
    G, p, st, it = ctx.forward_field(l, to_dev(kap), want_p=True)
    Gr, pr = oracle.forward_kappa(l, 7, kap, want_p=True)
    assert (host(st) == 0).all()
    assert rel_err(host(p), pr) < 1e-9


def test_forward_edge_cases():
    device()
    l = 4
    ctx = P.Context(3, 5, 10, 1.0, 0.3, 3, 0.01)
    case("forward N=0 and N=1")
    th = torch.zeros((0, 10), dtype=torch.float64, device="cuda:0")
    G = ctx.forward(l, th)
    assert G.shape == (0, 9)
    th1 = inputs.theta_batch(1, 1, 10)
    G1 = host(ctx.forward(l, to_dev(th1)))
    assert rel_err(G1, oracle.forward(l, 10, 1.0, 0.3, 3, th1)) < 1e-10
    case("forward level outside the context")
    with pytest.raises(P.Mls2mcError):
        ctx.forward(6, to_dev(th1))
    case("non-finite coefficient -> status 2")
    kap = inputs.kappa_batch(2, 3, oracle.n_elem(l))
    kap[1, 17] = np.nan
    G, p, st, it = ctx.forward_field(l, to_dev(kap))
    s = host(st)
    assert s[1] == 2 and s[0] == 0 and s[2] == 0


def test_forward_iteration_cap_reports_not_converged():
    device()
    l = 6
    case("max_iters=1 -> status 1")
    ctx = P.Context(l, l, 10, 1.0, 0.3, 3, 0.01, max_iters=1)
    th = inputs.theta_batch(3, 8, 10, scale=2.0)
    G, st, it = ctx.forward(l, to_dev(th), with_stats=True)
    assert (host(st) == 1).all() and (host(it) == 1).all()


@pytest.mark.parametrize("l,N,nsample", [(8, 600, 3), (9, 48, 1)])
def test_forward_full_size_sampled(l, N, nsample):
    """full-size levels: the oracle checks sampled particles one by one"""
    device()
    K, m = 100 if l == 8 else 200, 7 if l == 8 else 10
    corr = 0.3 if l == 8 else 0.1
    case(f"forward full-size l={l} N={N} K={K}")
    ctx = P.Context(l, l, K, 1.0, corr, m, 0.01)
    th = inputs.theta_batch(40 + l, N, K)
    G, st, it = ctx.forward(l, to_dev(th), with_stats=True)
    G = host(G)
    assert (host(st) == 0).all()
    idx = np.linspace(0, N - 1, nsample).astype(int)
    Gr = oracle.forward(l, K, 1.0, corr, m, th[idx])
    assert rel_err(G[idx], Gr) < 1e-10
    print(f"  iters mean {host(it).mean():.1f}")


def test_mixed_forward_field_parity():
    """FP32 inner MG-PCG + FP64 refinement: rel 1e-6 against the oracle given
    the same coefficients (the FP32-rounded kappa, promoted)."""
    device()
    for l in [3, 5, 7]:
        case(f"mixed forward_field l={l}")
        ctx = P.Context(l, l, 4, 1.0, 0.3, 5, 0.01, precision=P.MIXED)
        kap = inputs.kappa_batch(200 + l, 21, oracle.n_elem(l), spread=1.0)
        kap32 = kap.astype(np.float32).astype(np.float64)
        G, p, st, it = ctx.forward_field(l, to_dev(kap32), want_p=True)
        Gr, pr = oracle.forward_kappa(l, 5, kap32, want_p=True)
        assert (host(st) == 0).all()
        e = rel_err(host(p), pr)
        print(f"  rel err {e:.2e} inner iters {host(it).mean():.1f}")
        assert e < 1e-6


@pytest.mark.parametrize("l,K,N", [(5, 100, 130), (3, 10, 1), (7, 200, 77), (2, 33, 64), (4, 256, 65), (3, 300, 70)])
def test_mixed_bf16_field_error_bound(l, K, N):
    """BF16 KL GEMM with FP32 accumulation: |a_bf16 - a| is bounded by the
    rounding of theta and B to 8-bit mantissas (2^-8 relative each).  The
    cases cover K padded to 32 ... 256 (the column-tile kernel's one to eight
    32-wide k steps), K = 300 (beyond them: the 64 x 64 tile kernel), ragged
    row tiles (N = 1, 65, 77, 130) and a level with fewer elements than one
    column tile (h = 1/4: 32).  Each
    output element depends only on its row of theta, so the rows of a
    sub-batch are bitwise those of the whole batch."""
    device()
    case(f"bf16 kl_field l={l} K={K} N={N}")
    ctx = P.Context(l, l, K, 1.0, 0.3, 3, 0.01, precision=P.MIXED)
    th = inputs.theta_batch(9, N, K)
    kap32 = host(ctx.kl_field(l, to_dev(th), P.FIELD_KAPPA_F32)).astype(np.float64)
    B = oracle.kl_basis(l, K, 1.0, 0.3)
    a = th @ B
    bound = 2 * 2.0 ** -8 * (np.abs(th) @ np.abs(B)) + 1e-5 * np.abs(a) + 1e-6
    err = np.abs(np.log(kap32) - a)
    assert np.all(err <= bound)
    print(f"  max |a_bf16 - a| = {err.max():.3e}")
    sub = host(ctx.kl_field(l, to_dev(th[N // 2:]), P.FIELD_KAPPA_F32)).astype(np.float64)
    np.testing.assert_array_equal(sub, kap32[N // 2:])


@pytest.mark.parametrize("l,N", [(3, 64), (5, 64), (6, 32), (7, 16), (8, 8)])
def test_mixed_forward_error_against_oracle_per_level(l, N):
    """The whole mixed form (BF16 KL GEMM, FP32 solver with FP64 residual
    replacement) against the FP64 oracle on prior draws, K = 100, 49
    observations.  Its error is the BF16 field's.  Rounding theta and B to
    BF16 (relative error up to u = 2^-8 each, independent from term to term)
    perturbs an element's log-field with standard deviation
    sigma_e = sqrt(2 u^2 / 3 * sum_k (theta_k B_ke)^2), so kappa by a factor
    exp(+-sigma_e); the observations, weighted averages of p, move by less
    than the largest such factor: |dG| / |G| <= 6 max_e sigma_e (8 sigma_e is
    the Gaussian tail of the largest of 10^5 elements).  Besides that
    derived bound, the measured errors (3.3e-3 at most, 1.6e-3 from h = 1/128
    on, on the box this was written on) must stay below 5e-3."""
    device()
    K, m = 100, 7
    case(f"mixed forward vs oracle l={l} N={N}")
    ctx = P.Context(l, l, K, 1.0, 0.3, m, 0.002, precision=P.MIXED)
    th = inputs.theta_batch(600 + l, N, K)
    G, st, it = ctx.forward(l, to_dev(th), with_stats=True)
    Gr = oracle.forward(l, K, 1.0, 0.3, m, th)
    B = oracle.kl_basis(l, K, 1.0, 0.3)
    sig = np.sqrt(2.0 * (2.0 ** -8) ** 2 / 3.0 * ((th * th) @ (B * B)).max(1))
    Gh = host(G)
    assert (host(st) == 0).all()
    err = np.abs(Gh - Gr).max(1) / np.abs(Gr).max(1)
    print(f"  h=1/{1 << l}: max rel G error {err.max():.2e} (median {np.median(err):.2e}), "
          f"derived bound 6 sigma {6 * sig.max():.2e}, mean iters {host(it).mean():.1f}")
    assert np.all(err <= 6 * sig)
    assert err.max() < 5e-3


LDS_MAX = 160 * 1024 - 1024  # gfx950: 160 KiB of LDS per workgroup, 1 KiB kept for static arrays


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("l", [4, 5, 6, 7])
def test_solver_schedules_give_identical_results(l, prec):
    """LDS residency (none; coarse levels only; coarse levels and some or all
    fine arrays) and the persistent grid change where the arrays live and
    which workgroup solves which particle, not the arithmetic: bitwise equal
    results for a fixed block size.  Other block sizes split the reductions
    differently (rounding only)."""
    device()
    N = 50 if l <= 6 else 12
    ctx = P.Context(l, l, 20, 1.0, 0.3, 5, 0.01, precision=P.MIXED if prec == "mixed" else P.FP64)
    th = to_dev(inputs.theta_batch(61, N, 20))
    for block in (256, 512):
        outs = []
        for grid, lds in [(0, 0), (7, -1), (N, 0), (13, -1), (5, 20000), (9, 81920), (N, LDS_MAX)]:
            case(f"schedule l={l} {prec} grid={grid} block={block} lds={lds}")
            ctx.set_launch(l, grid, block, 1, lds)
            G, st, it = ctx.forward(l, th, with_stats=True)
            assert host(st).max() == 0
            outs.append((host(G), host(it)))
        for G, it in outs[1:]:
            np.testing.assert_array_equal(G, outs[0][0])
            np.testing.assert_array_equal(it, outs[0][1])
        if block == 256:
            G256 = outs[0][0]
    assert rel_err(outs[0][0], G256) < (1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("form", ["fp64", "mixed", "flow"])
def test_forward_chunks_are_seamless(form):
    """At h = 1/512 a forward splits its batch into 2 GiB coefficient chunks
    (512 particles in FP64, 1024 in FP32).  A particle's result does not
    depend on the batch it is solved in, so a batch of 520 (FP64) or 1030
    (FP32) must equal, bit for bit, a separate batch of its last particles,
    across the chunk boundary."""
    device()
    l, K, m = 9, 20, 5
    N = 1030 if form == "mixed" else 520
    case(f"forward chunks l={l} {form} N={N}")
    kw = dict(precision=P.MIXED) if form == "mixed" else dict(bc=P.BC_FLOW_CELL) if form == "flow" else {}
    ctx = P.Context(l, l, K, 1.0, 0.3, m, 0.01, **kw)
    th = to_dev(inputs.theta_batch(13, N, K))
    G, st, it = ctx.forward(l, th, with_stats=True)
    assert host(st).max() == 0
    tail = N - 15
    G2, st2, it2 = ctx.forward(l, th[tail:].contiguous(), with_stats=True)
    np.testing.assert_array_equal(host(G)[tail:], host(G2))
    np.testing.assert_array_equal(host(it)[tail:], host(it2))


@pytest.mark.parametrize("l,N", [(8, 40), (9, 12)])
def test_column_walk_instances_parity(l, N):
    """Blocks that the row width divides (256, 512 and 1024 threads at
    h = 1/256; 512 and 1024 at h = 1/512) run the solver instances whose CG
    stencil pass walks columns, in one, two or four bands of rows.  FP64 and
    mixed, on the same FP32-representable coefficients: sampled particles
    against the oracle (rel 1e-10 and 1e-6), and all particles against a
    row-loop launch with half the row width (rel 1e-9 and 1e-5: only the
    summation order of the inner products differs)."""
    device()
    n = 1 << l
    kap = inputs.kappa_batch(60 + l, N, oracle.n_elem(l), spread=1.0)
    kap32 = kap.astype(np.float32).astype(np.float64)
    idx = [N - 1] if l == 9 else [0, N - 1]
    Gr = oracle.forward_kappa(l, 7, kap32[idx])
    for prec, tol, tol_rl in ((P.FP64, 1e-10, 1e-9), (P.MIXED, 1e-6, 1e-5)):
        ctx = P.Context(l, l, 4, 1.0, 0.3, 7, 0.01, precision=prec)
        case(f"column walk l={l} row loop block={n // 2} precision={prec}")
        ctx.set_launch(l, N, n // 2, 1, -1)
        G_rl, p, st, it = ctx.forward_field(l, to_dev(kap32))
        assert host(st).max() == 0
        for block in (n, 2 * n, 4 * n):
            if block > 1024:
                continue
            case(f"column walk l={l} block={block} precision={prec}")
            ctx.set_launch(l, N, block, 1, -1)
            G, p, st, it = ctx.forward_field(l, to_dev(kap32))
            assert host(st).max() == 0
            assert rel_err(host(G)[idx], Gr) < tol
            assert rel_err(host(G), host(G_rl)) < tol_rl
        ctx.close()


@pytest.mark.parametrize("prec", [P.MIXED, P.FP64])
def test_walked_levels_after_smaller_levels_in_one_context(prec):
    """The solver's workspace is shared by the levels of a context, so a
    solve on h = 1/256 or 1/512 finds the words that smaller levels' solves
    left in it, FP64 words among them in the mixed form.  Boundary entries
    that the walks never write must not reach the results: after solves on
    h = 1/128 and 1/256 in the same context, every particle converges and G
    equals, bit for bit, that of a fresh context for the same level."""
    device()
    K, m = 200, 10
    th = to_dev(inputs.theta_batch(77, 4096, K))
    shape = (256, 1024, 1, -1)
    case(f"walked levels after smaller ones, precision={prec}")
    ctx = P.Context(7, 9, K, 1.0, 0.1, m, 0.001, precision=prec)
    for lv in (7, 8, 9):
        ctx.set_launch(lv, *shape)
    outs = {}
    for lv, N in ((7, 4096), (8, 4096), (9, 2048)):
        G, st, it = ctx.forward(lv, th[:N].contiguous(), with_stats=True)
        bad = int((host(st) != 0).sum())
        print(f"  h=1/{1 << lv}: {bad} of {N} not converged")
        assert bad == 0
        outs[lv] = host(G)
    for lv, N in ((8, 4096), (9, 2048)):
        fresh = P.Context(lv, lv, K, 1.0, 0.1, m, 0.001, precision=prec)
        fresh.set_launch(lv, *shape)
        G, st, it = fresh.forward(lv, th[:N].contiguous(), with_stats=True)
        assert (host(st) == 0).all()
        np.testing.assert_array_equal(outs[lv], host(G))
        fresh.close()
    ctx.close()


@pytest.mark.parametrize("l,m", [(3, 7), (6, 7), (8, 7), (5, 32)])
def test_observations_without_the_field(l, m):
    """The FP64 forward without p_out gathers G = Obs x step by step from the
    search directions and never stores x; with p_out it keeps x.  Same
    iteration counts, the same G up to rounding, and the field-free G
    matches the oracle on sampled particles."""
    device()
    N = 40  # m = 32: 1024 observations, more than the threads of a workgroup
    case(f"forward_field G with and without the field l={l} m={m} N={N}")
    ctx = P.Context(l, l, 4, 1.0, 0.3, m, 0.01)
    kap = inputs.kappa_batch(320 + l, N, oracle.n_elem(l), spread=1.0)
    G0, _, st0, it0 = ctx.forward_field(l, to_dev(kap), want_p=False)
    G1, p1, st1, it1 = ctx.forward_field(l, to_dev(kap), want_p=True)
    assert (host(st0) == 0).all() and (host(st1) == 0).all()
    np.testing.assert_array_equal(host(it0), host(it1))
    assert rel_err(host(G0), host(G1)) < 1e-13
    idx = [0, N - 1]
    assert rel_err(host(G0)[idx], oracle.forward_kappa(l, m, kap[idx])) < 1e-10
