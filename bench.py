"""Benchmark of the MLS^2MC hot path on one MI355X.

Default workload (synthetic, seeded): the largest single-GPU configuration,
MLS^2MC on levels h = 1/16 .. 1/512 (l = 4..9; 261,121 unknowns per
particle on the finest level), K = 200 separable-exponential KL terms
(sigma^2 = 1, correlation length 0.1), 100 observations on a 10x10 interior
grid, sigma_n = 0.001, J = 8192 particles, 5 pCN steps per stage with
s = 0.5, ESS target 0.5 J.

A step is one SMC sub-step on the finest level over all J particles:
adaptive next temperature (log-sum-exp weights), integer-CDF resampling,
gather, and one pCN move whose J proposals go through the KL field GEMM,
the multigrid-PCG solve, the observations, the potential and the
acceptance (a configured stage makes five such moves).  The timed steps run
the plain FP64 form; `value` = forward solves/s at h = 1/512 inside them.
Extra fields: the same step in the mixed-precision form, per-level
forward solves/s of both forms with the mixed form's error against the FP64
path, time-to-posterior of plain FP64 against mixed precision + surrogate
(with the paper's RelErr and RelMisfit of each posterior mean), the roofline
of the h = 1/512 solver kernel measured live with HIP events recorded by the
library on its launch stream, and the CPU oracle on a bounded sample with
an extrapolated CPU time-to-posterior.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic bytes per fine-level unknown per PCG iteration of the
# multigrid-PCG: PCG vector work + V(1,1) cycle, each array read once and
# written once per sweep, coarse levels included (293 B with the iterate
# x); each further smoothing step per side adds two sweeps reading x, b and
# the two weight arrays and writing x, over all levels (2 x 5 x 8 x 4/3 =
# 106.7 B).  The FP64 forward gathers the observations from the search
# directions and never stores x, so its model drops x's read and write
# (16 B: 277 B).  The mixed form keeps its iterate; half of 293 B with its
# FP32 inner arrays.
def b_iter(nu, fp32=False):
    if fp32:
        return (293.0 + 106.7 * (max(1, nu) - 1)) / 2
    return 277.0 + 106.7 * (max(1, nu) - 1)


B_ITER_FP64 = b_iter(1)
B_ITER_MIXED = b_iter(1, True)
PMC_H64 = os.path.join(ROOT, "profiles", "solve_h64_K50_J1000_pmc.md")
PMC_H512 = os.path.join(ROOT, "profiles", "solve_h512_K200_J8192_pmc.md")
TUNED_DIR = os.path.join(ROOT, "paper_1709_09763_amd", "tuned")
TUNED_H64 = os.path.join(TUNED_DIR, "mi355x_h8-64_K50_J1000.json")
TUNED_H512 = os.path.join(TUNED_DIR, "mi355x_h16-512_K200_J8192.json")


def solver_sha():
    """first 16 hex digits of sha256 over the solver's sources"""
    import hashlib
    h = hashlib.sha256()
    for f in ("solver.hip", "common.h"):
        h.update(open(os.path.join(ROOT, "paper_1709_09763_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(summary, shape, form="fp64"):
    """HBM bytes per solver launch from a committed rocprofv3 counter
    summary, or None once the solver source or the launch shape
    (grid, block, nu, lds) differs from the one measured.  The summary
    holds lines `solver_source_sha256_16: ...`, `launch_shape[_<form>]:
    g,b,nu,lds` and `traffic_bytes_per_launch[_<form>]: B`."""
    try:
        txt = open(summary).read()
    except OSError:
        return None
    vals = {}
    for ln in txt.splitlines():
        if ":" in ln and ln.split(":", 1)[0].strip().replace("_", "").isalnum():
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("solver_source_sha256_16", "") != solver_sha():
        return None
    suf = "" if form == "fp64" and "launch_shape" in vals else f"_{form}"
    if vals.get("launch_shape" + suf, "") != ",".join(str(v) for v in shape):
        return None
    try:
        return float(vals["traffic_bytes_per_launch" + suf])
    except (KeyError, ValueError):
        return None


def device_key():
    """the GPU's architecture and compute-unit count (its marketing name can
    differ between runs, e.g. under a profiler)"""
    import torch
    pr = torch.cuda.get_device_properties(0)
    return f"{pr.gcnArchName.split(':')[0]}:{pr.multi_processor_count}cu"


def tuned_matches(rec):
    """a tuned-shape record applies when it was made on this kind of device
    for this solver source"""
    import torch
    same_dev = (rec.get("device_key") == device_key() if "device_key" in rec
                else rec.get("device") == torch.cuda.get_device_name(0))
    return same_dev and rec.get("solver_source_sha256_16") == solver_sha()


def load_tuned(path, ctxs):
    """apply committed launch shapes {form: {level: shape}} when they were
    tuned on this device for this solver source; returns the path or None"""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if not tuned_matches(rec):
        return None
    for form, c in ctxs.items():
        for lv, sh in rec.get(form, {}).items():
            c.set_launch(int(lv), sh["grid"], sh["block"], sh.get("nu", 0), sh.get("lds", 0))
    return path


def cpu_model():
    """the host CPU's model name (what lscpu reports, read from /proc/cpuinfo)"""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


WL = dict(name="mls2mc h=1/8..1/64 K=50 Nobs=25 J=1000", l_min=3, l_max=6, K=50, m=5,
          sigma_n=0.005, J=1000, corr=0.3, n_mcmc=5, s_pcn=0.5, tau_star=1.0)


def solve_bytes(l, nobs, particles, iters, b_iter):
    n = 1 << l
    M = (n - 1) ** 2
    n_e = 2 * n * n
    setup = 8 * n_e + (4.0 / 3.0) * 2 * 2 * n * (n - 1) * 8
    return particles * (setup + 8 * 4 * nobs) + iters * b_iter * M


def flow_solve_bytes(l, nobs, particles, iters, nu):
    """streaming model of the flow-cell solver's fused passes, per fine
    unknown and PCG iteration: p = z + beta p_old with q = A p 48 B (FP64
    weights), the r update with the first red sweep 48 B (the forward keeps
    no iterate: its observations are gathered step by step), and on the fine
    level, whose V-cycle reads FP32 weights, 120 + 128 (nu - 1) B (black
    sweep 32, restriction of the red residuals 24, black and red sweeps 64)
    plus the coarse correction: a prolongation pass of 18 B below h = 1/128,
    2 B of coarse values read inside the first black sweep from there on;
    the coarse levels (FP64 weights) add a third of 170 + 160 (nu - 1) B;
    per solve also the coefficients, the zeroed slot (nine fine arrays and
    four per coarse level) and the observations"""
    n = 1 << l
    M = (n - 1) * (n + 1)
    correction = 18 if l < 7 else 2
    b_iter = 48 + 48 + 120 + correction + 128 * (nu - 1) + (170 + 160 * (nu - 1)) / 3.0
    fsz = (n + 1) * (n + 3)
    slot = 9 * fsz + 4 * fsz / 3.0 + 2 * n * n / 3.0
    return particles * (8 * 2 * n * n + 8 * slot + 32 * nobs) + iters * b_iter * M


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(l, K, m, corr, budget_s=15.0):
    """the oracle as it stands, timed on the host cores on chunks of prior
    draws until the time budget is used"""
    import numpy as np

    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rng = np.random.default_rng(7)
    chunk = 4 * cores
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        oracle.forward(l, K, 1.0, corr, m, rng.standard_normal((chunk, K)), nthreads=cores)
        n += chunk
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="forward solves/s", cores=cores, kind="oracle", cpu=cpu_model(),
                sample=f"{n} forward solves at h=1/{1 << l}, K={K} from the prior, in chunks of "
                       f"{chunk} (KL field, generic P1 assembly, banded Cholesky, observation), "
                       f"OpenMP over particles, {dt:.1f}s")


def cpu_levels(levels, K, m, corr, budget_s=2.0, single_core_level=None):
    """The oracle (KL field, generic P1 assembly, banded Cholesky, observation)
    on the host cores, one solve per thread: per level, chunks of `cores`
    prior draws until `budget_s` is used (at least one chunk); optionally one
    solve on one thread at `single_core_level`.  Returns {level: solves/s on
    all cores}, the single-core solves/s, cores and the CPU model."""
    import numpy as np

    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rng = np.random.default_rng(7)
    rates, samples = {}, {}
    for lv in levels:
        n, t0 = 0, time.perf_counter()
        while n == 0 or time.perf_counter() - t0 < budget_s:
            oracle.forward(lv, K, 1.0, corr, m, rng.standard_normal((cores, K)), nthreads=cores)
            n += cores
        dt = time.perf_counter() - t0
        rates[lv] = n / dt
        samples[lv] = f"{n} solves in {dt:.1f}s"
        log(f"cpu oracle h=1/{1 << lv}: {rates[lv]:.3g} solves/s ({samples[lv]})")
    single = None
    if single_core_level is not None:
        t0 = time.perf_counter()
        oracle.forward(single_core_level, K, 1.0, corr, m, rng.standard_normal((1, K)), nthreads=1)
        single = 1.0 / (time.perf_counter() - t0)
        log(f"cpu oracle single core h=1/{1 << single_core_level}: {single:.3g} solves/s")
    return rates, samples, single, cores, cpu_model()


def rel_misfit(G, y):
    """the paper's relative misfit |Gamma^{-1/2}(y - G)|^2 / |Gamma^{-1/2} y|^2
    (Sec. 5.1; Gamma = sigma_n^2 I cancels)"""
    import numpy as np
    G, y = np.asarray(G, dtype=np.float64), np.asarray(y, dtype=np.float64)
    return float(((y - G) ** 2).sum() / (y ** 2).sum())


def rel_err_paper(mean, truth, lam):
    """relative error of a posterior mean with Lambda^{1/2} weights (Sec. 5.1)"""
    import numpy as np
    w = np.sqrt(lam)
    return float(np.abs(w * (mean - truth)).sum() / np.abs(w * truth).sum())


def tune_levels(ctx, levels, J):
    out = {}
    for lv in levels:
        ms, (g, b, nu, lds) = ctx.autotune(lv, min(J, 512 if lv >= 7 else J))
        out[f"h=1/{1 << lv}"] = dict(grid=g, block=b, nu=nu, lds=lds, ms=round(ms, 4))
    return out


W4 = dict(name="mls2mc h=1/16..1/512 K=200 corr=0.1 Nobs=100 sigma_n=0.001 J=8192", l_min=4, l_max=9, K=200,
          m=10, sigma_n=0.001, J=8192, corr=0.1, n_mcmc=5, s_pcn=0.5, tau_star=1.0)


def run_summary(r, mean, th_true, lam, misfit):
    """the fields every time-to-posterior record carries"""
    return dict(seconds=round(r["seconds"], 3), stages=r["n_stages"],
                solves={str(i): v for i, v in enumerate(r["solves"]) if v},
                accept_rate=round(r["accepted"] / max(1, r["proposed"]), 5), log_Z=r["log_Z"],
                rel_err_vs_truth=round(rel_err_paper(mean, th_true, lam), 4), rel_misfit=round(misfit, 6),
                mean_pcg_iters=round(r["iters_total"] / max(1, sum(r["solves"])), 2),
                not_converged=r["not_converged"])


def leg_largest_stage(args):
    """The default benchmark (see the module docstring)."""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    W = W4
    K, m, J, L, sn = W["K"], W["m"], W["J"], W["l_max"], W["sigma_n"]
    lv_all = range(W["l_min"], L + 1)
    ctx = P.Context(W["l_min"], L, K, 1.0, W["corr"], m, sn)
    ctxm = P.Context(W["l_min"], L, K, 1.0, W["corr"], m, sn, precision=P.MIXED)
    nobs = ctx.nobs
    lam = ctx.kl_eigenvalues()
    rng = np.random.default_rng(99)
    th_true = rng.standard_normal(K)
    y = ctx.forward(L, torch.tensor(th_true[None, :], device=dev))[0]
    y = (y + sn * torch.tensor(rng.standard_normal(nobs), device=dev)).contiguous()
    extras = {}
    src = None if args.retune else load_tuned(args.tuned or TUNED_H512, {"fp64": ctx, "mixed": ctxm})
    if src:
        extras["solver_launch_source"] = os.path.relpath(src, ROOT)
        log(f"solver launch shapes from {src}")
    elif not args.no_autotune:
        tuned = {}
        for name, c in (("fp64", ctx), ("mixed", ctxm)):
            tuned[name] = {}
            for lv in lv_all:
                ms, (g, b, nu, lds) = c.autotune(lv, 512)
                tuned[name][str(lv)] = dict(grid=g, block=b, nu=nu, lds=lds)
                log(f"autotuned {name} h=1/{1 << lv}: {tuned[name][str(lv)]} {ms:.3f} ms")
        if args.save_tuned:
            json.dump({"device": torch.cuda.get_device_name(0), "device_key": device_key(), "workload": W["name"],
                       "solver_source_sha256_16": solver_sha(), **tuned}, open(args.save_tuned, "w"), indent=1)
        extras["solver_launch_source"] = "autotuned in this run on 512 prior draws per level"
    else:
        extras["solver_launch_source"] = "library defaults"
    extras["solver_launch"] = {name: {f"h=1/{1 << lv}": list(c.get_launch(lv)) for lv in lv_all}
                               for name, c in (("fp64", ctx), ("mixed", ctxm))}

    thp = None
    if not args.no_extras:
        # ---- time-to-posterior, plain FP64 against mixed precision + surrogate:
        # at the configured fixed pCN step, and with the step adapted between
        # stages (an extension; with sigma_n = 0.001 the fixed step's
        # acceptance collapses on the fine levels, so the chains barely move
        # there).  One untimed short run of each form first.
        sur = dict(surrogate=True, sur_collect_max_level=6, sur_da_min_level=7, sur_pairs=20480, sur_epochs=15,
                   sur_hidden=256)
        ctx.run(y, 256, seed=1)
        ctxm.run(y, 256, seed=1, **sur)
        torch.cuda.synchronize()
        extras["time_to_posterior_s"] = {}
        for step_rule, adapt in (("fixed_step", False), ("adapted_step", True)):
            runs = {}
            for name, c, kw in (("plain_fp64", ctx, {}), ("mixed_surrogate", ctxm, sur)):
                r = c.run(y, J, J_tilde=100, tau_star=W["tau_star"], n_mcmc=W["n_mcmc"], s_pcn=W["s_pcn"], seed=31,
                          s_adapt=adapt, **kw)
                th = r["theta"]
                mean = th.mean(0, keepdim=True).contiguous()
                Gm = ctx.forward(L, mean)[0]
                rec = run_summary(r, mean[0].cpu().numpy(), th_true, lam,
                                  rel_misfit(Gm.cpu().numpy(), y.cpu().numpy()))
                if kw:
                    rec.update(surrogate_train_s=round(r["sur_train_seconds"], 3),
                               stage1_pass_frac=round(r["stage1_passed"] / max(1, r["da_proposed"]), 4),
                               surrogate_err_over_sigma_n=dict(mean=round(r["sur_err_mean"], 4),
                                                               max=round(r["sur_err_max"], 4),
                                                               solves_judged=r["sur_err_count"]))
                runs[name] = (r, rec, mean[0].cpu().numpy())
                log(f"time-to-posterior {step_rule} {name}: {rec}")
                if name == "plain_fp64" and not adapt:
                    thp = th.contiguous()
                    solves_fp64 = r["solves"]
            extras["time_to_posterior_s"][step_rule] = {k: v[1]["seconds"] for k, v in runs.items()}
            extras["time_to_posterior_s"][step_rule]["speedup_mixed_surrogate_vs_plain_fp64"] = round(
                runs["plain_fp64"][1]["seconds"] / runs["mixed_surrogate"][1]["seconds"], 3)
            extras[f"run_{step_rule}"] = {k: v[1] for k, v in runs.items()}
            extras[f"run_{step_rule}"]["rel_err_between_forms"] = round(
                rel_err_paper(runs["mixed_surrogate"][2], runs["plain_fp64"][2], lam), 4)

        # ---- per-level forward solves/s of both forms on J prior draws, and the
        # mixed form's error against the FP64 path (itself rel 1e-10 of the oracle)
        per = {"fp64": {}, "mixed": {}, "mixed_rel_err_vs_fp64": {}}
        thr = torch.tensor(rng.standard_normal((J, K)), device=dev)
        for lv in lv_all:
            Gs = {}
            for name, c in (("fp64", ctx), ("mixed", ctxm)):
                c.forward(lv, thr[:512].contiguous())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Gs[name] = c.forward(lv, thr)
                torch.cuda.synchronize()
                per[name][f"h=1/{1 << lv}"] = round(J / (time.perf_counter() - t0), 1)
            d = (Gs["mixed"] - Gs["fp64"]).abs().amax(1) / Gs["fp64"].abs().amax(1)
            per["mixed_rel_err_vs_fp64"][f"h=1/{1 << lv}"] = dict(max=float(d.max()), median=float(d.median()))
            log(f"per-level h=1/{1 << lv}: fp64 {per['fp64'][f'h=1/{1 << lv}']}, mixed {per['mixed'][f'h=1/{1 << lv}']}"
                f" solves/s, mixed rel err max {float(d.max()):.2e}")
        extras["forward_solves_per_s_by_level"] = per

    # ---- state for the timed steps: the FP64 run's posterior particles at h = 1/512
    theta = thp if thp is not None else torch.tensor(rng.standard_normal((J, K)), device=dev)

    def make_state(c):
        th = theta.clone()
        G = c.forward(L, th)
        return dict(theta=th, G=G, phi=c.loglik(G, y), theta2=torch.empty_like(th), G2=torch.empty_like(G),
                    phi2=torch.empty_like(G[:, 0]).contiguous())

    beta0 = 0.5

    def step(c, S, k):
        out3, logw, w = c.next_step(S["phi"], 1.0, beta0, J / (1 + W["tau_star"] ** 2))
        u = c.philox(99, 3, k, 0, J, normal=False)
        anc = c.resample(w, u)
        P.mls2mc_gather(c.h, anc, S["theta"], S["theta2"])
        P.mls2mc_gather(c.h, anc, S["G"], S["G2"])
        P.mls2mc_gather(c.h, anc, S["phi"].view(-1, 1), S["phi2"].view(-1, 1))
        for a, b in (("theta", "theta2"), ("G", "G2"), ("phi", "phi2")):
            S[a], S[b] = S[b], S[a]
        xi = c.philox(99, 4, k, 0, J * K, normal=True).view(J, K)
        uu = c.philox(99, 5, k, 0, J, normal=False)
        c.pcn_step(L, L, 0.75, 1.0, W["s_pcn"], S["theta"], S["G"], None, S["phi"], None, y, xi, uu)

    def timed(c, steps, warmup):
        S = make_state(c)
        for k in range(warmup):
            step(c, S, 10_000 + k)
        torch.cuda.synchronize()
        c.profile(True)
        t0 = time.perf_counter()
        for k in range(steps):
            step(c, S, k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        c.profile(False)
        return dt, c.profile_read(P.PROF_SOLVE, L), c.profile_read(P.PROF_GEMM, L)

    # mixed form first (not the driver's step count), then the timed FP64 steps
    msteps = max(2, min(args.steps, 5))
    dtm, psm, pgm = timed(ctxm, msteps, 1)
    extras["mixed_stage"] = dict(steps=msteps, solves_per_s=round(msteps * J / dtm, 1),
                                 ms_per_step=round(dtm / msteps * 1e3, 3),
                                 solver_avg_ms=round(psm["ms"] / max(1, psm["launches"]), 3),
                                 mean_pcg_iters=round(psm["iters"] / max(1, psm["items"]), 3),
                                 solver_algorithmic_GBs=round(
                                     solve_bytes(L, nobs, psm["items"], psm["iters"],
                                                 b_iter(ctxm.get_launch(L)[2], True)) / (psm["ms"] * 1e-3) / 1e9, 1))
    gflop = 2.0 * pgm["items"] * K * (2 << (2 * L))
    extras["mixed_stage"]["kl_gemm_bf16_tflops"] = round(gflop / max(pgm["ms"] * 1e-3, 1e-12) / 1e12, 2)
    log(f"mixed stage {extras['mixed_stage']}")
    dt, ps, pg = timed(ctx, args.steps, args.warmup)
    value = args.steps * J / dt
    nu_l = ctx.get_launch(L)[2]
    alg = solve_bytes(L, nobs, ps["items"], ps["iters"], b_iter(nu_l))
    avg_ms = ps["ms"] / max(1, ps["launches"])
    achieved = alg / ps["launches"] / (avg_ms * 1e-3) / 1e9 if ps["launches"] else 0.0
    traffic = measured_traffic(PMC_H512, ctx.get_launch(L), "fp64")
    gflop = 2.0 * pg["items"] * K * (2 << (2 * L))
    extras["solver_kernel"] = dict(launches=ps["launches"], particles_per_launch=ps["items"] / max(1, ps["launches"]),
                                   avg_ms=round(avg_ms, 4), mean_pcg_iters=round(ps["iters"] / max(1, ps["items"]), 3),
                                   share_of_step_time=round(ps["ms"] * 1e-3 / dt, 3))
    extras["kl_gemm"] = dict(launches=pg["launches"], avg_ms=round(pg["ms"] / max(1, pg["launches"]), 4),
                             tflops=round(gflop / max(pg["ms"] * 1e-3, 1e-12) / 1e12, 3),
                             frac_of_fp64_peak=round(gflop / max(pg["ms"] * 1e-3, 1e-12) / 1e12 / FP64_PEAK_TFLOPS, 4))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
            "algorithmic_bytes_per_launch": round(alg / max(1, ps["launches"]), 0),
            "kernel": "solve_kernel (h=1/512, FP64)", "launch_shape": list(ctx.get_launch(L))}
    if traffic:
        roof["measured_rate_GBs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        roof["traffic_over_algorithmic"] = round(traffic / (alg / ps["launches"]), 3)
    cpu = None
    if not args.no_cpu_baseline:
        rates, samples, single, cores, model = cpu_levels(
            [L] if args.no_extras else list(lv_all), K, m, W["corr"], budget_s=1.5,
            single_core_level=None if args.quick_cpu else L)
        cpu = dict(value=rates[L], unit="forward solves/s (h=1/512)", cores=cores, kind="oracle",
                   sample=f"{samples[L]} at h=1/512 (K=200, corr 0.1, prior draws; KL field, generic P1 assembly, "
                          f"banded Cholesky, observation), one solve per thread on all {cores} threads",
                   cpu_model=model, single_core_solves_per_s=single,
                   by_level={f"h=1/{1 << lv}": round(v, 3) for lv, v in rates.items()})
        if not args.no_extras:
            t_cpu = sum(n / rates[lv] for lv, n in enumerate(solves_fp64) if n and lv in rates)
            cpu["time_to_posterior_s_extrapolated"] = round(t_cpu, 1)
            cpu["extrapolation"] = ("sum over levels of the plain FP64 GPU run's solve count times the oracle's "
                                    "measured seconds per solve on all cores")
        log(f"cpu baseline {cpu}")
    out = {
        "metric": "forward solves/s per level; MLS²MC time-to-posterior, plain vs surrogate+FP32",
        "value": round(value, 2),
        "unit": "forward solves/s (h=1/512, inside SMC sub-steps)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["name"], "levels": "h=1/16..1/512", "K": K, "corr_len": W["corr"], "n_obs": nobs,
                   "J": J, "sigma_n": sn, "pcn_step": W["s_pcn"],
                   "step": "one SMC sub-step at h=1/512 over all J particles: next_step, resample, gather, one pCN "
                           "move (KL GEMM + MG-PCG solve + observation + potential + accept); a configured stage "
                           "makes 5 such moves"},
        "roofline": roof,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out))


def leg_fast(args):
    """h=1/8..1/256, K=100, 49 obs, sigma_n=0.002, J=4096: time-to-posterior of
    the plain FP64 form and of the mixed-precision + surrogate form.  With
    --seeds R > 1 each form runs R times; the posterior-mean error of every
    run is then measured against the mean over all 2R runs as well as
    against the true parameter."""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    K, m, sn, J, lmin, lmax = 100, 7, 0.002, 4096, 3, 8
    rng = np.random.default_rng(77)
    th_true = rng.standard_normal(K)
    ctx = P.Context(lmin, lmax, K, 1.0, 0.3, m, sn)
    lam = ctx.kl_eigenvalues()
    y = ctx.forward(lmax, torch.tensor(th_true[None, :], device=dev))[0]
    y = (y + sn * torch.tensor(rng.standard_normal(m * m), device=dev)).contiguous()
    tuned = tune_levels(ctx, range(lmin, lmax + 1), J)
    log(f"fast leg: tuned fp64 {tuned}")
    ctxm = P.Context(lmin, lmax, K, 1.0, 0.3, m, sn, precision=P.MIXED)
    tune_levels(ctxm, range(lmin, lmax + 1), J)
    seeds = [21 + i for i in range(max(1, args.seeds))]
    runs = {"plain_fp64": [], "mixed_surrogate": []}
    if args.fp64_surrogate:
        runs["fp64_surrogate"] = []
    for sd in seeds:
        r = ctx.run(y, J, seed=sd, s_adapt=args.s_adapt)
        runs["plain_fp64"].append(dict(
            seconds=r["seconds"], stages=r["n_stages"], solves={str(i): v for i, v in enumerate(r["solves"]) if v},
            mean=r["theta"].cpu().numpy().mean(0), log_Z=r["log_Z"],
            stage_acc_rate=[round(float(a), 4) for a in r["stage_acc_rate"]]))
        rm = ctxm.run(y, J, seed=sd, surrogate=True, sur_collect_max_level=6, sur_da_min_level=7,
                      sur_pairs=20480, sur_epochs=15, sur_hidden=256, s_adapt=args.s_adapt)
        runs["mixed_surrogate"].append(dict(
            seconds=rm["seconds"], stages=rm["n_stages"], solves={str(i): v for i, v in enumerate(rm["solves"]) if v},
            mean=rm["theta"].cpu().numpy().mean(0), log_Z=rm["log_Z"],
            surrogate_train_s=round(rm["sur_train_seconds"], 3),
            stage1_pass_frac=rm["stage1_passed"] / max(1, rm["da_proposed"]),
            stage_acc_rate=[round(float(a), 4) for a in rm["stage_acc_rate"]]))
        if args.fp64_surrogate:
            rs = ctx.run(y, J, seed=sd, surrogate=True, sur_collect_max_level=6, sur_da_min_level=7,
                         sur_pairs=20480, sur_epochs=15, sur_hidden=256, s_adapt=args.s_adapt)
            runs["fp64_surrogate"].append(dict(
                seconds=rs["seconds"], stages=rs["n_stages"],
                solves={str(i): v for i, v in enumerate(rs["solves"]) if v},
                mean=rs["theta"].cpu().numpy().mean(0), log_Z=rs["log_Z"],
                surrogate_train_s=round(rs["sur_train_seconds"], 3),
                stage1_pass_frac=rs["stage1_passed"] / max(1, rs["da_proposed"]),
                stage_acc_rate=[round(float(a), 4) for a in rs["stage_acc_rate"]]))
        log(f"seed {sd}: plain {runs['plain_fp64'][-1]['seconds']:.3f} s, "
            f"mixed+surrogate {runs['mixed_surrogate'][-1]['seconds']:.3f} s"
            + (f", fp64+surrogate {runs['fp64_surrogate'][-1]['seconds']:.3f} s" if args.fp64_surrogate else ""))
    pooled = np.mean([d["mean"] for v in runs.values() for d in v], axis=0)
    out = {}
    for name, v in runs.items():
        o = dict(v[0])
        o.pop("mean")
        o["seconds"] = round(float(np.median([d["seconds"] for d in v])), 3)
        o["seconds_all"] = [round(d["seconds"], 3) for d in v]
        o["rel_err_vs_truth"] = [rel_err_paper(d["mean"], th_true, lam) for d in v]
        o["log_Z_all"] = [d["log_Z"] for d in v]
        if len(v) > 1:
            o["rel_err_vs_pooled_mean"] = [rel_err_paper(d["mean"], pooled, lam) for d in v]
        out[name] = o
        log(f"{name} {o}")
    out["rel_err_between_forms"] = rel_err_paper(np.mean([d["mean"] for d in runs["mixed_surrogate"]], 0),
                                                 np.mean([d["mean"] for d in runs["plain_fp64"]], 0), lam)
    print(json.dumps({
        "metric": "MLS²MC time-to-posterior, plain vs surrogate+FP32",
        "value": out["mixed_surrogate"]["seconds"], "unit": "s (mixed precision + surrogate)",
        "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "bf16/f32/f64",
        "data": "synthetic", "speedup_vs_plain_fp64": round(out["plain_fp64"]["seconds"] / out["mixed_surrogate"]["seconds"], 3),
        "config": {"workload": "mls2mc h=1/8..1/256 K=100 Nobs=49 sigma_n=0.002 J=4096",
                   "pcn_step": "adapted" if args.s_adapt else "fixed 0.5", "seeds": seeds}, **out}))


def interp_time_at(err_target, errs, times):
    """time at which a form reaches err_target, by linear interpolation of
    log time against log error along its (N-sweep) curve; extrapolated from
    the two nearest points when the target lies outside the curve"""
    import numpy as np
    e, t = np.log(np.asarray(errs, float)), np.log(np.asarray(times, float))
    order = np.argsort(e)
    e, t = e[order], t[order]
    x = np.log(err_target)
    inside = bool(e[0] <= x <= e[-1])
    if inside:
        return float(np.exp(np.interp(x, e, t))), False
    i = 0 if x < e[0] else len(e) - 2
    slope = (t[i + 1] - t[i]) / (e[i + 1] - e[i]) if e[i + 1] != e[i] else 0.0
    return float(np.exp(t[i] + slope * (x - e[i]))), True


def leg_equal_error(args):
    """Equal posterior-mean error on h=1/8..1/256, K=100 (corr 0.3), 49 obs,
    sigma_n=0.002: a reference posterior mean from plain FP64 runs with 4 x
    4096 particles (--ref-seeds of them, averaged); then, for plain FP64 and
    for mixed precision + surrogate, --seeds runs at every N of --sizes.
    Reports per form and N the mean and standard error of the paper's RelErr
    (Sec. 5.1, Lambda^{1/2}-weighted l1) against the reference mean and
    against the truth, RelMisfit, the log-evidence spread and the median time
    to posterior; and the fast form's time at the plain form's error at the
    largest N (log-log interpolation along its N sweep)."""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    K, m, sn, lmin, lmax, corr = 100, 7, 0.002, 3, 8, 0.3
    sizes = [int(v) for v in args.sizes.split(",")]
    rng = np.random.default_rng(77)
    th_true = rng.standard_normal(K)
    ctx = P.Context(lmin, lmax, K, 1.0, corr, m, sn)
    lam = ctx.kl_eigenvalues()
    y = ctx.forward(lmax, torch.tensor(th_true[None, :], device=dev))[0]
    y = (y + sn * torch.tensor(rng.standard_normal(m * m), device=dev)).contiguous()
    y_h = y.cpu().numpy()
    ctxm = P.Context(lmin, lmax, K, 1.0, corr, m, sn, precision=P.MIXED)
    tune_levels(ctx, range(lmin, lmax + 1), max(sizes))
    tune_levels(ctxm, range(lmin, lmax + 1), max(sizes))
    step = dict(s_adapt=args.s_adapt, s_pcn=0.5)
    sur = dict(surrogate=True, sur_collect_max_level=6, sur_da_min_level=7, sur_pairs=20480, sur_epochs=15,
               sur_hidden=256)
    ctx.run(y, 256, seed=1, **step)
    ctxm.run(y, 256, seed=1, **step, **sur)

    def misfit(mean):
        G = ctx.forward(lmax, torch.tensor(mean[None, :], device=dev))[0]
        return rel_misfit(G.cpu().numpy(), y_h)

    # reference posterior mean
    Jref = 4 * max(sizes)
    ref_means, ref_t = [], []
    for i in range(args.ref_seeds):
        r = ctx.run(y, Jref, seed=1000 + i, **step)
        ref_means.append(r["theta"].mean(0).cpu().numpy())
        ref_t.append(r["seconds"])
        log(f"reference run {i}: J={Jref} {r['seconds']:.2f}s stages {r['n_stages']}")
    ref = np.mean(ref_means, axis=0)
    ref_spread = [rel_err_paper(mu, ref, lam) for mu in ref_means]
    out = {"reference": dict(J=Jref, runs=args.ref_seeds, seconds=[round(t, 3) for t in ref_t],
                             rel_err_of_each_run_vs_their_mean=[round(v, 4) for v in ref_spread],
                             rel_err_vs_truth=round(rel_err_paper(ref, th_true, lam), 4),
                             rel_misfit=round(misfit(ref), 6))}
    seeds = [21 + i for i in range(args.seeds)]
    forms = (("plain_fp64", ctx, {}), ("mixed_surrogate", ctxm, sur))
    for name, c, kw in forms:
        out[name] = {}
        for N in sizes:
            rows = []
            for sd in seeds:
                r = c.run(y, N, seed=sd, **step, **kw)
                mu = r["theta"].mean(0).cpu().numpy()
                row = dict(seconds=r["seconds"], rel_err_ref=rel_err_paper(mu, ref, lam),
                           rel_err_truth=rel_err_paper(mu, th_true, lam), rel_misfit=misfit(mu), log_Z=r["log_Z"],
                           solves=sum(r["solves"]))
                if kw:
                    row.update(stage1_pass=r["stage1_passed"] / max(1, r["da_proposed"]),
                               sur_err_mean=r["sur_err_mean"], sur_err_max=r["sur_err_max"],
                               train_s=r["sur_train_seconds"])
                rows.append(row)
            R = len(rows)
            agg = dict(runs=R, seconds_median=round(float(np.median([q["seconds"] for q in rows])), 4),
                       seconds_all=[round(q["seconds"], 3) for q in rows])
            for k in ("rel_err_ref", "rel_err_truth", "rel_misfit"):
                v = np.array([q[k] for q in rows])
                agg[k] = dict(mean=round(float(v.mean()), 5),
                              se=round(float(v.std(ddof=1) / np.sqrt(R)) if R > 1 else 0.0, 5))
            lz = np.array([q["log_Z"] for q in rows])
            agg["log_Z"] = dict(mean=round(float(lz.mean()), 3), sd=round(float(lz.std(ddof=1)) if R > 1 else 0.0, 3))
            agg["solves_mean"] = float(np.mean([q["solves"] for q in rows]))
            if kw:
                for k in ("stage1_pass", "sur_err_mean", "sur_err_max", "train_s"):
                    agg[k] = round(float(np.mean([q[k] for q in rows])), 4)
            out[name][str(N)] = agg
            log(f"{name} N={N}: t {agg['seconds_median']}s RelErr(ref) {agg['rel_err_ref']} "
                f"RelErr(truth) {agg['rel_err_truth']}")
    Nmax = str(max(sizes))
    e_plain = out["plain_fp64"][Nmax]["rel_err_ref"]["mean"]
    t_plain = out["plain_fp64"][Nmax]["seconds_median"]
    errs = [out["mixed_surrogate"][str(N)]["rel_err_ref"]["mean"] for N in sizes]
    times = [out["mixed_surrogate"][str(N)]["seconds_median"] for N in sizes]
    t_fast, extrap = interp_time_at(e_plain, errs, times)
    out["equal_error"] = dict(plain_error=e_plain, plain_seconds=t_plain, fast_seconds_at_plain_error=round(t_fast, 4),
                              extrapolated=extrap, speedup=round(t_plain / t_fast, 3))
    # the same runs read per particle count: time ratio and the difference of
    # the forms' mean errors with its standard error (a difference within two
    # standard errors is not resolved by this many seeds)
    by_size = {}
    for N in sizes:
        a, b = out["plain_fp64"][str(N)], out["mixed_surrogate"][str(N)]
        row = dict(time_ratio_plain_over_fast=round(a["seconds_median"] / b["seconds_median"], 3))
        for k in ("rel_err_ref", "rel_err_truth", "rel_misfit"):
            row[k + "_fast_minus_plain"] = dict(diff=round(b[k]["mean"] - a[k]["mean"], 5),
                                                se=round(float(np.hypot(a[k]["se"], b[k]["se"])), 5))
        by_size[str(N)] = row
    out["by_size"] = by_size
    # and at equal time: the plain form's error interpolated (log-log along
    # its N sweep) at the fast form's time for the largest N
    e_pl = [out["plain_fp64"][str(N)]["rel_err_ref"]["mean"] for N in sizes]
    t_pl = [out["plain_fp64"][str(N)]["seconds_median"] for N in sizes]
    tf = out["mixed_surrogate"][Nmax]["seconds_median"]
    lt, le = np.log(t_pl), np.log(e_pl)
    order = np.argsort(lt)
    e_at = float(np.exp(np.interp(np.log(tf), lt[order], le[order])))
    out["equal_time"] = dict(fast_seconds=tf, fast_error=out["mixed_surrogate"][Nmax]["rel_err_ref"]["mean"],
                             plain_error_at_that_time=round(e_at, 5),
                             plain_time_range_covers=bool(lt.min() <= np.log(tf) <= lt.max()))
    log(f"equal error {out['equal_error']}")
    print(json.dumps({
        "metric": "MLS²MC time-to-posterior at equal posterior-mean error, plain FP64 vs surrogate+FP32",
        "value": out["equal_error"]["speedup"], "unit": "time ratio plain / fast at the plain form's RelErr",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64 vs bf16/f32/f64",
        "data": "synthetic",
        "config": {"workload": "mls2mc h=1/8..1/256 K=100 Nobs=49 sigma_n=0.002", "sizes": sizes, "seeds": seeds,
                   "pcn_step": "adapted" if args.s_adapt else "fixed 0.5"}, **out}))


def leg_compare(args):
    """The paper's comparison on the h=1/8..1/64, K=50, 25 obs, J=1000
    workload: MLS^2MC, MLS^2MC with the adaptive maximum level (tau_min =
    0.001), multilevel bridging, and single-level SMC on h=1/64, each with
    pCN and with the random-walk kernel (step 2.38/sqrt(K)); cost in the
    paper's normalised units C_l = 4^(l - 6), over --seeds runs"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    W = WL
    K, m, J = W["K"], W["m"], W["J"]
    rng = np.random.default_rng(2024)
    ctx = P.Context(W["l_min"], W["l_max"], K, 1.0, W["corr"], m, W["sigma_n"])
    th_true = rng.standard_normal(K)
    y = ctx.forward(W["l_max"], torch.tensor(th_true[None, :], device=dev))[0]
    y = (y + W["sigma_n"] * torch.tensor(rng.standard_normal(ctx.nobs), device=dev)).contiguous()
    ctx1 = P.Context(W["l_max"], W["l_max"], K, 1.0, W["corr"], m, W["sigma_n"])
    lam = ctx.kl_eigenvalues()
    forms = {"mls2mc": (ctx, {}), "mls2mc_adaptive_max_level": (ctx, dict(tau_min=1e-3)),
             "multilevel_bridging": (ctx, dict(scheme=P.SCHEME_MLB)), "single_level_smc": (ctx1, {})}
    seeds = [11 + i for i in range(max(1, args.seeds))]
    out = {}
    for kname, kern, step in (("pcn", P.KERNEL_PCN, 0.5), ("rwm", P.KERNEL_RWM, 2.38 / np.sqrt(K))):
        for name, (c, kw) in forms.items():
            rows = []
            for sd in seeds:
                r = c.run(y, J, J_tilde=100, seed=sd, kernel=kern, s_pcn=step, **kw)
                cost = sum(v * 4.0 ** (lv - W["l_max"]) for lv, v in enumerate(r["solves"]))
                rows.append(dict(seconds=r["seconds"], cost=cost, log_Z=r["log_Z"], final_level=r["final_level"],
                                 stages=r["n_stages"], accept=r["accepted"] / max(1, r["proposed"]),
                                 rel_err=rel_err_paper(r["theta"].cpu().numpy().mean(0), th_true, lam)))
            agg = {k: float(np.mean([q[k] for q in rows])) for k in rows[0]}
            agg["log_Z_sd"] = float(np.std([q["log_Z"] for q in rows], ddof=1)) if len(rows) > 1 else None
            out[f"{name}_{kname}"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in agg.items()}
            log(f"compare {name} {kname}: {out[f'{name}_{kname}']}")
    base = out["single_level_smc_pcn"]["cost"]
    print(json.dumps({
        "metric": "MLS²MC vs comparison schemes (cost in normalised solves C_l = 4^(l-6))",
        "value": round(base / out["mls2mc_pcn"]["cost"], 3), "unit": "cost ratio single-level SMC / MLS²MC (pCN)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["name"], "seeds": seeds}, **out}))


def leg_levels(args):
    """Forward solves/s for every level h=1/8..1/512 at N = 1024 and 8192,
    K=100, corr 0.3, 49 obs, FP64 and mixed, on prior draws and on
    posterior particles of an h=1/8..1/256 run (sigma_n=0.002); launch
    shapes autotuned per level on 512 prior draws"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    K, m, sn, lmin, lmax = 100, 7, 0.002, 3, 9
    rng = np.random.default_rng(4)
    prior = torch.tensor(rng.standard_normal((8192, K)), device=dev)
    ctx = P.Context(lmin, lmax, K, 1.0, 0.3, m, sn)
    th_true = torch.tensor(rng.standard_normal((1, K)), device=dev)
    y = (ctx.forward(8, th_true)[0] + sn * torch.tensor(rng.standard_normal(m * m), device=dev)).contiguous()
    ctx_run = P.Context(lmin, 8, K, 1.0, 0.3, m, sn)
    post = ctx_run.run(y, 4096, seed=5, s_adapt=True)["theta"]
    post = torch.cat([post, post]).contiguous()  # 8192 posterior particles (two copies of 4096)
    res = {}
    for pname, prec in (("fp64", P.FP64), ("mixed", P.MIXED)):
        c = P.Context(lmin, lmax, K, 1.0, 0.3, m, sn, precision=prec)
        for lv in range(lmin, lmax + 1):
            c.autotune(lv, 512)
            row = {}
            for src, th in (("prior", prior), ("posterior", post)):
                for N in (1024, 8192):
                    x = th[:N].contiguous()
                    c.forward(lv, x[:256].contiguous())
                    torch.cuda.synchronize()
                    c.profile(True)
                    t0 = time.perf_counter()
                    G, st, it = c.forward(lv, x, with_stats=True)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    c.profile(False)
                    ps = c.profile_read(P.PROF_SOLVE, lv)
                    alg = solve_bytes(lv, m * m, ps["items"], ps["iters"], b_iter(c.get_launch(lv)[2], prec == P.MIXED))
                    row[f"{src}_N{N}"] = dict(solves_per_s=round(N / dt, 1),
                                              mean_iters=round(float(it.float().mean().item()), 2),
                                              solver_algorithmic_GBs=round(alg / (ps["ms"] * 1e-3) / 1e9, 1),
                                              converged=int((st == 0).sum().item()))
            res[f"{pname}_h=1/{1 << lv}"] = dict(launch=list(c.get_launch(lv)), **row)
            log(f"levels {pname} h=1/{1 << lv}: " + ", ".join(f"{k} {v['solves_per_s']}" for k, v in row.items()))
        c.close()
    print(json.dumps({
        "metric": "forward solves/s per level", "value": res["fp64_h=1/64"]["prior_N1024"]["solves_per_s"],
        "unit": "forward solves/s (h=1/64, N=1024, prior draws)", "n_gpus": 1, "higher_is_better": True,
        "vs_baseline": None, "dtype": "f64 / mixed", "data": "synthetic",
        "config": {"workload": "h=1/8..1/512, K=100, corr 0.3, Nobs=49, N in {1024, 8192}"}, **res}))


def leg_kl(args):
    """The KL field kernels alone (a = theta B_l with the exp epilogue) at the
    configured shapes: FP64 MFMA and BF16 MFMA (FP32 accumulation), N rows,
    timed with HIP events on the stream they run on, 5 launches each"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    res = {}
    for l, K, corr, N in ((9, 200, 0.1, 2048), (8, 100, 0.3, 4096), (6, 50, 0.3, 1000)):
        ne = 2 * 4 ** l
        th = torch.tensor(np.random.default_rng(l).standard_normal((N, K)), device=dev)
        for form, prec, kind in (("fp64", P.FP64, P.FIELD_KAPPA_F64), ("bf16", P.MIXED, P.FIELD_KAPPA_F32)):
            c = P.Context(l, l, K, 1.0, corr, 7, 0.01, precision=prec)
            out = torch.empty((N, ne), dtype=torch.float64 if form == "fp64" else torch.float32, device=dev)
            P.mls2mc_kl_field(c.h, l, th, out, kind)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record()
            for _ in range(reps):
                P.mls2mc_kl_field(c.h, l, th, out, kind)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            flops = 2.0 * N * K * ne
            Kp = (K + 31) // 32 * 32
            # algorithmic bytes: theta read, basis read once, kappa written
            byts = 8.0 * N * K + (8.0 * K * ne + 8.0 * N * ne if form == "fp64" else 2.0 * Kp * ne + 4.0 * N * ne)
            res[f"{form}_h=1/{1 << l}_K{K}_N{N}"] = dict(
                ms=round(ms, 3), tflops=round(flops / ms / 1e9, 1), algorithmic_GBs=round(byts / ms / 1e6, 1),
                write_GBs=round((8.0 if form == "fp64" else 4.0) * N * ne / ms / 1e6, 1))
            log(f"kl {form} h=1/{1 << l} K={K} N={N}: {ms:.3f} ms, {flops / ms / 1e9:.1f} TFLOP/s, "
                f"{byts / ms / 1e6:.0f} GB/s")
            del out
            c.close()
    print(json.dumps({
        "metric": "KL field TFLOP/s", "value": res["bf16_h=1/512_K200_N2048"]["tflops"], "unit": "TFLOP/s",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64 / bf16 (f32 acc.)",
        "data": "synthetic", "config": {"workload": "KL field h=1/512 K=200, h=1/256 K=100, h=1/64 K=50"},
        **res}))


def leg_batched(args):
    """32 instances, seeds 0..31, J ~ U{256..4096}, finest h in {1/64, 1/128,
    1/256}, K=100, 49 obs, sigma_n=0.002: fused rounds with HIP graphs"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    K, m, sn, lmin, lmax = 100, 7, 0.002, 3, 8
    ctx = P.Context(lmin, lmax, K, 1.0, 0.3, m, sn)
    specs = []
    for seed in range(32):
        g = np.random.default_rng(1000 + seed)
        J = int(g.integers(256, 4097))
        lm = int(g.choice([6, 7, 8]))
        th_true = torch.tensor(g.standard_normal((1, K)), device=dev)
        y = ctx.forward(lm, th_true)[0] + sn * torch.tensor(g.standard_normal(m * m), device=dev)
        specs.append(dict(J=J, l_max=lm, y=y.contiguous(), seed=seed))
    t0 = time.perf_counter()
    out = ctx.run_batch([dict(d) for d in specs], use_graphs=True)
    dt = time.perf_counter() - t0
    solves = sum(sum(o["solves"]) for o in out)
    res = dict(seconds=round(dt, 3), total_particles=sum(d["J"] for d in specs), total_solves=solves,
               graphs=out[0]["graphs_launched"],
               finest_levels={str(k): sum(1 for d in specs if d["l_max"] == k) for k in (6, 7, 8)})
    log(f"batched {res}")
    if args.batched_sequential:
        t0 = time.perf_counter()
        for d in specs:
            ctx.run(d["y"], d["J"], seed=d["seed"])
        torch.cuda.synchronize()
        res["sequential_seconds"] = round(time.perf_counter() - t0, 3)
    print(json.dumps({
        "metric": "MLS²MC time-to-posterior (32 uneven instances, fused)", "value": res["seconds"], "unit": "s",
        "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "32 instances J~U{256..4096}, finest h in {1/64,1/128,1/256}, K=100, Nobs=49"},
        **res}))


def leg_largest_run(args):
    """h=1/16..1/512, K=200 (correlation length 0.1), 100 obs, sigma_n=0.001,
    J=8192: full MLS^2MC, plain FP64 vs mixed precision + surrogate"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    K, m, sn, J, lmin, lmax = 200, 10, 0.001, 8192, 4, 9
    rng = np.random.default_rng(99)
    th_true = rng.standard_normal(K)
    out = {}
    for name, prec, sur in (("plain_fp64", P.FP64, False), ("mixed_surrogate", P.MIXED, True)):
        ctx = P.Context(lmin, lmax, K, 1.0, 0.1, m, sn, precision=prec)
        lam = ctx.kl_eigenvalues()
        if name == "plain_fp64":
            y = ctx.forward(lmax, torch.tensor(th_true[None, :], device=dev))[0]
            y = (y + sn * torch.tensor(rng.standard_normal(m * m), device=dev)).contiguous()
        tune_levels(ctx, range(lmin, lmax + 1), J)
        kw = dict(surrogate=True, sur_collect_max_level=6, sur_da_min_level=7, sur_pairs=20480,
                  sur_epochs=15, sur_hidden=256) if sur else {}
        r = ctx.run(y, J, seed=31, s_adapt=args.s_adapt, **kw)
        mean = r["theta"].cpu().numpy().mean(0)
        out[name] = dict(seconds=round(r["seconds"], 3), stages=r["n_stages"],
                         solves={str(i): v for i, v in enumerate(r["solves"]) if v},
                         rel_err_vs_truth=rel_err_paper(mean, th_true, lam), log_Z=r["log_Z"],
                         accept_rate=r["accepted"] / max(1, r["proposed"]),
                         stage_levels=r["stage_level"].tolist(),
                         stage_acc_rate=[round(float(a), 4) for a in r["stage_acc_rate"]])
        if sur:
            out[name].update(surrogate_train_s=round(r["sur_train_seconds"], 3),
                             stage1_pass_frac=r["stage1_passed"] / max(1, r["da_proposed"]))
        out[name]["mean"] = mean
        log(f"{name} {dict((k, v) for k, v in out[name].items() if k != 'mean')}")
        ctx.close()
    out["rel_err_between_forms"] = rel_err_paper(out["mixed_surrogate"].pop("mean"), out["plain_fp64"].pop("mean"), lam)
    print(json.dumps({
        "metric": "MLS²MC time-to-posterior, plain vs surrogate+FP32", "value": out["mixed_surrogate"]["seconds"],
        "unit": "s (mixed precision + surrogate)", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
        "dtype": "bf16/f32/f64", "data": "synthetic",
        "speedup_vs_plain_fp64": round(out["plain_fp64"]["seconds"] / out["mixed_surrogate"]["seconds"], 3),
        "config": {"workload": "mls2mc h=1/16..1/512 K=200 corr=0.1 Nobs=100 sigma_n=0.001 J=8192",
                   "pcn_step": "adapted" if args.s_adapt else "fixed 0.5"}, **out}))


def leg_largest(args):
    """h=1/512, K=200 (correlation length 0.1), 100 obs, J=8192: forward solves/s
    of plain FP64 and mixed precision batches"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    K, m, sn, J, l = 200, 10, 0.001, 8192, 9
    rng = np.random.default_rng(5)
    th = torch.tensor(rng.standard_normal((J, K)), device=dev)
    res = {}
    for name, prec in (("fp64", P.FP64), ("mixed", P.MIXED)):
        ctx = P.Context(l, l, K, 1.0, 0.1, m, sn, precision=prec)
        tuned = tune_levels(ctx, [l], 512)
        ctx.forward(l, th[:1024].contiguous())
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        G, st, it = ctx.forward(l, th, with_stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.profile(False)
        ps = ctx.profile_read(P.PROF_SOLVE, l)
        alg = solve_bytes(l, 100, ps["items"], ps["iters"], b_iter(ctx.get_launch(l)[2], prec == P.MIXED))
        res[name] = dict(launch=tuned[f"h=1/{1 << l}"], solves_per_s=round(J / dt, 1), seconds=round(dt, 3),
                         mean_iters=float(it.float().mean().item()), converged=int((st == 0).sum().item()),
                         solver_algorithmic_GBs=round(alg / (ps["ms"] * 1e-3) / 1e9, 1))
        log(f"largest {name} {res[name]}")
        ctx.close()
    print(json.dumps({
        "metric": "forward solves/s per level", "value": res["fp64"]["solves_per_s"], "unit": "forward solves/s (h=1/512)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "h=1/512 K=200 corr=0.1 Nobs=100 J=8192 forward batch"}, **res}))


def leg_matern(args):
    """Matern (nu = 3/2) priors of the paper's elliptic examples (Sec. 5,
    Examples 5.1 and 5.3; source f = 1 and the homogeneous Dirichlet problem
    of the main path): KL build time (Nystrom eigenpairs and the basis at every
    level), forward solves/s at the finest level, and one MLS^2MC run"""
    import numpy as np
    import torch

    import paper_1709_09763_amd as P
    dev = torch.device("cuda:0")
    cfgs = [("example_5_1", dict(lmin=3, lmax=7, K=10, lam=0.65, m=5, sn=0.07, J=1000)),
            ("example_5_3", dict(lmin=4, lmax=8, K=320, lam=0.1, m=7, sn=0.045, J=1000, bc=P.BC_FLOW_CELL))]
    out = {}
    for name, c in cfgs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = P.Context(c["lmin"], c["lmax"], c["K"], 1.0, c["lam"], c["m"], c["sn"], cov=P.COV_MATERN32,
                        bc=c.get("bc", P.BC_DIRICHLET))
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        lam = ctx.kl_eigenvalues()
        rng = np.random.default_rng(71)
        l, K = c["lmax"], c["K"]
        tune_levels(ctx, range(c["lmin"], l + 1), c["J"])
        th = torch.tensor(rng.standard_normal((1024, K)), device=dev)
        ctx.forward(l, th[:256].contiguous())
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        G, st, it = ctx.forward(l, th, with_stats=True)
        torch.cuda.synchronize()
        fwd = 1024 / (time.perf_counter() - t0)
        ctx.profile(False)
        ps = ctx.profile_read(P.PROF_SOLVE, l)
        flow = c.get("bc", P.BC_DIRICHLET) == P.BC_FLOW_CELL
        nu_l = ctx.get_launch(l)[2] or 1
        alg = (flow_solve_bytes(l, ctx.nobs, ps["items"], ps["iters"], nu_l) if flow
               else solve_bytes(l, ctx.nobs, ps["items"], ps["iters"], b_iter(nu_l)))
        solver_gbs = round(alg / (ps["ms"] * 1e-3) / 1e9, 1)
        th_true = rng.standard_normal(K)
        y = ctx.forward(l, torch.tensor(th_true[None, :], device=dev))[0]
        y = (y + c["sn"] * torch.tensor(rng.standard_normal(ctx.nobs), device=dev)).contiguous()
        r = ctx.run(y, c["J"], seed=13)
        mean = r["theta"].cpu().numpy().mean(0)
        out[name] = dict(config=dict((k, v) for k, v in c.items()), kl_build_s=round(build, 3),
                         variance_fraction=round(float(lam.sum()), 4),
                         problem="flow cell" if flow else "Dirichlet, f = 1",
                         forward_solves_per_s=round(fwd, 1), mean_iters=float(it.float().mean().item()),
                         solver_ms=round(ps["ms"], 3), solver_algorithmic_GBs=solver_gbs,
                         converged=int((st == 0).sum().item()),
                         run=dict(seconds=round(r["seconds"], 3), stages=r["n_stages"],
                                  solves={str(i): v for i, v in enumerate(r["solves"]) if v},
                                  rel_err_vs_truth=rel_err_paper(mean, th_true, lam), log_Z=r["log_Z"],
                                  accept_rate=r["accepted"] / max(1, r["proposed"])))
        log(f"matern {name} {out[name]}")
        ctx.close()
    print(json.dumps({
        "metric": "Matern-prior KL build and forward solves/s", "value": out["example_5_3"]["forward_solves_per_s"],
        "unit": "forward solves/s (flow cell, h=1/256, K=320 Matern prior)", "n_gpus": 1, "higher_is_better": True,
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Matern 3/2 priors of Examples 5.1 (lam 0.65, K 10, h 1/8..1/128, Dirichlet, f=1) "
                               "and 5.3 (lam 0.1, K 320, h 1/16..1/256, flow cell), Nystrom grid 64"}, **out}))


def copy_calibration(gib=2.0):
    """plain device copy of known size, for scaling rocprofv3 byte counters"""
    import torch
    n = int(gib * (1 << 30) // 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip per-level and time-to-posterior")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even when the committed shapes match this device and solver")
    ap.add_argument("--tuned", default=None, help="JSON of solver launch shapes to use instead of tuning")
    ap.add_argument("--save-tuned", default=None, help="write the tuned launch shapes to this JSON")
    ap.add_argument("--workload", default="largest-stage",
                    choices=["largest-stage", "stages-h64", "fast", "batched", "largest", "largest-run", "compare",
                             "levels", "matern", "equal-error", "kl"],
                    help="largest-stage: the default benchmark; others: the extra workloads")
    ap.add_argument("--quick-cpu", action="store_true", help="skip the single-core oracle solve at h=1/512")
    ap.add_argument("--seeds", type=int, default=1, help="fast / equal-error: independent runs per form (and N)")
    ap.add_argument("--ref-seeds", type=int, default=4, help="equal-error: runs averaged for the reference mean")
    ap.add_argument("--sizes", default="1024,2048,4096", help="equal-error: particle counts swept")
    ap.add_argument("--fp64-surrogate", action="store_true",
                    help="fast: also run the surrogate form with the FP64 solver")
    ap.add_argument("--s-adapt", action="store_true",
                    help="fast / largest-run: adapt the pCN step between stages (an extension)")
    ap.add_argument("--batched-sequential", action="store_true",
                    help="batched workload: also time the instances one after another")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the particle axis would shard across GPUs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1709_09763_amd as P

    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload != "stages-h64":
        {"largest-stage": leg_largest_stage, "fast": leg_fast, "batched": leg_batched, "largest": leg_largest,
         "largest-run": leg_largest_run, "compare": leg_compare, "levels": leg_levels,
         "matern": leg_matern, "equal-error": leg_equal_error, "kl": leg_kl}[args.workload](args)
        return
    dev = torch.device("cuda:0")
    W = WL
    K, m, J, l = W["K"], W["m"], W["J"], W["l_max"]
    ctx = P.Context(W["l_min"], W["l_max"], K, 1.0, W["corr"], m, W["sigma_n"])
    nobs = ctx.nobs
    rng = np.random.default_rng(2024)
    th_true = torch.tensor(rng.standard_normal((1, K)), device=dev)
    y = ctx.forward(l, th_true)[0] + W["sigma_n"] * torch.tensor(rng.standard_normal(nobs), device=dev)
    y = y.contiguous()

    extras = {}
    shapes, shapes_m = {}, {}
    tuned_file = args.tuned
    if tuned_file is None and not args.retune and not args.no_autotune and os.path.exists(TUNED_H64):
        rec = json.load(open(TUNED_H64))
        if tuned_matches(rec):
            tuned_file = TUNED_H64  # the committed shapes were tuned on this device for this solver
    ctxm = P.Context(W["l_min"], W["l_max"], K, 1.0, W["corr"], m, W["sigma_n"], precision=P.MIXED)
    if tuned_file:
        rec = json.load(open(tuned_file))
        shapes = {int(k): v for k, v in rec["fp64"].items()}
        shapes_m = {int(k): v for k, v in rec.get("mixed", {}).items()}
        for c, sh_ in ((ctx, shapes), (ctxm, shapes_m)):
            for lv, sh in sh_.items():
                c.set_launch(lv, sh["grid"], sh["block"], sh.get("nu", 0), sh.get("lds", 0))
        extras["solver_launch"] = {f"h=1/{1 << lv}": sh for lv, sh in shapes.items()}
        extras["solver_launch_source"] = os.path.relpath(tuned_file, ROOT)
        log(f"solver launch shapes from {tuned_file}")
    elif not args.no_autotune:
        tuned = {}
        for c, sh_, key in ((ctx, shapes, "fp64"), (ctxm, shapes_m, "mixed")):
            for lv in range(W["l_min"], W["l_max"] + 1):
                ms, (g, b, nu, lds) = c.autotune(lv, J)
                sh_[lv] = dict(grid=g, block=b, nu=nu, lds=lds)
                if key == "fp64":
                    tuned[f"h=1/{1 << lv}"] = dict(grid=g, block=b, nu=nu, lds=lds, ms=round(ms, 4))
        extras["autotuned_solver_launch"] = tuned
        log(f"autotuned {tuned}")
        if args.save_tuned:
            json.dump({"device": torch.cuda.get_device_name(0), "device_key": device_key(), "workload": W["name"],
                       "solver_source_sha256_16": solver_sha(),
                       "fp64": {str(k): v for k, v in shapes.items()},
                       "mixed": {str(k): v for k, v in shapes_m.items()}}, open(args.save_tuned, "w"), indent=1)
    if not args.no_extras:
        # time-to-posterior, plain FP64 (one untimed warm run first)
        ctx.run(y, 200, seed=1)
        torch.cuda.synchronize()
        r = ctx.run(y, J, J_tilde=100, tau_star=W["tau_star"], n_mcmc=W["n_mcmc"], s_pcn=W["s_pcn"], seed=11)
        thp = r["theta"].cpu().numpy()
        extras["time_to_posterior_fp64_s"] = round(r["seconds"], 4)
        extras["run_fp64"] = dict(stages=r["n_stages"], solves={str(i): v for i, v in enumerate(r["solves"]) if v},
                                  log_Z=r["log_Z"], mean_pcg_iters=r["iters_total"] / max(1, sum(r["solves"])),
                                  accept_rate=r["accepted"] / max(1, r["proposed"]))
        log(f"time-to-posterior fp64 {r['seconds']:.3f}s stages {r['n_stages']}")
        ctxm.run(y, 200, seed=1)
        rm = ctxm.run(y, J, J_tilde=100, tau_star=W["tau_star"], n_mcmc=W["n_mcmc"], s_pcn=W["s_pcn"], seed=11)
        extras["time_to_posterior_mixed_s"] = round(rm["seconds"], 4)
        thm = rm["theta"].cpu().numpy()
        extras["run_mixed"] = dict(stages=rm["n_stages"], log_Z=rm["log_Z"],
                                   posterior_mean_rel_diff_vs_fp64=float(
                                       np.abs(thm.mean(0) - thp.mean(0)).sum() / np.abs(thp.mean(0)).sum()))
        log(f"time-to-posterior mixed {rm['seconds']:.3f}s")
        # per-level throughput of plain forward batches (J particles)
        per = {}
        th = torch.tensor(rng.standard_normal((J, K)), device=dev)
        for lv in range(W["l_min"], W["l_max"] + 1):
            ctx.forward(lv, th)
            torch.cuda.synchronize()
            reps = 5
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.forward(lv, th)
            torch.cuda.synchronize()
            per[f"h=1/{1 << lv}"] = round(reps * J / (time.perf_counter() - t0), 1)
        extras["forward_solves_per_s_by_level"] = per
        log(f"per-level {per}")

    # ---- state for the timed stages: posterior-like particles at level 6
    theta = torch.tensor(rng.standard_normal((J, K)), device=dev)
    if not args.no_extras:
        theta = torch.tensor(thp, device=dev)
    G = ctx.forward(l, theta)
    phi = ctx.loglik(G, y)
    theta2, G2, phi2 = torch.empty_like(theta), torch.empty_like(G), torch.empty_like(phi)
    stream = torch.cuda.current_stream()
    beta0 = 0.5

    def step(k):
        nonlocal theta, G, phi, theta2, G2, phi2
        out3, logw, w = ctx.next_step(phi, 1.0, beta0, J / (1 + W["tau_star"] ** 2))
        u = ctx.philox(99, 3, k, 0, J, normal=False)
        anc = ctx.resample(w, u)
        P.mls2mc_gather(ctx.h, anc, theta, theta2)
        P.mls2mc_gather(ctx.h, anc, G, G2)
        P.mls2mc_gather(ctx.h, anc, phi.view(-1, 1), phi2.view(-1, 1))
        theta, theta2, G, G2, phi, phi2 = theta2, theta, G2, G, phi2, phi
        for s in range(W["n_mcmc"]):
            xi = ctx.philox(99, 4, k, s, J * K, normal=True).view(J, K)
            uu = ctx.philox(99, 5, k, s, J, normal=False)
            ctx.pcn_step(l, l, 0.75, 1.0, W["s_pcn"], theta, G, None, phi, None, y, xi, uu)

    for k in range(args.warmup):
        step(10_000 + k)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(False)
    ps = ctx.profile_read(P.PROF_SOLVE, l)
    pg = ctx.profile_read(P.PROF_GEMM, l)
    solves = args.steps * W["n_mcmc"] * J
    value = solves / dt
    nu_l = ctx.get_launch(l)[2]
    alg = solve_bytes(l, nobs, ps["items"], ps["iters"], b_iter(nu_l))
    avg_ms = ps["ms"] / max(1, ps["launches"])
    achieved = alg / ps["launches"] / (avg_ms * 1e-3) / 1e9 if ps["launches"] else 0.0
    gemm_flops = 2.0 * pg["items"] * K * (2 << (2 * l))
    extras["solver_kernel"] = dict(launches=ps["launches"], avg_ms=round(avg_ms, 4),
                                   mean_pcg_iters=ps["iters"] / max(1, ps["items"]),
                                   share_of_step_time=round(ps["ms"] * 1e-3 / dt, 3))
    extras["kl_gemm"] = dict(launches=pg["launches"], avg_ms=round(pg["ms"] / max(1, pg["launches"]), 4),
                             tflops=round(gemm_flops / max(pg["ms"] * 1e-3, 1e-12) / 1e12, 3),
                             frac_of_fp64_peak=round(gemm_flops / max(pg["ms"] * 1e-3, 1e-12) / 1e12 / FP64_PEAK_TFLOPS, 4))
    traffic = measured_traffic(PMC_H64, ctx.get_launch(l))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(l, K, m, W["corr"])
        log(f"cpu baseline {cpu['value']:.1f} solves/s on {cpu['cores']} cores")
    out = {
        "metric": "forward solves/s per level; MLS²MC time-to-posterior, plain vs surrogate+FP32",
        "value": round(value, 2),
        "unit": "forward solves/s (h=1/64, inside SMC stages)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["name"], "levels": "h=1/8..1/64", "K": K, "n_obs": nobs, "J": J,
                   "sigma_n": W["sigma_n"], "step": "one SMC stage at h=1/64: next_step, resample, "
                   "gather, 5 pCN steps (KL GEMM + MG-PCG solve + observation + potential)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "algorithmic_bytes_per_launch": round(alg / max(1, ps["launches"]), 0),
                     "kernel": "solve_kernel (h=1/64, FP64)", "launch_shape": list(ctx.get_launch(l))},
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
