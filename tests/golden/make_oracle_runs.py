"""Writes oracle_runs.json: whole oracle sampler runs (Sec. 4.4, the final
update scheme) at the configured problem sizes, stored so that the GPU
parity tests compare against them without re-running the slow CPU sampler.

Every value comes from oracle/ alone: the data y = G_lmax(theta*) + sigma_n
eta from the oracle's forward map, then the oracle's sampler on the same
Philox streams the library draws.  Run from the repository root:

    python tests/golden/make_oracle_runs.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from tests import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")


def _batch_case(J, lmax, seed):
    K, m, sn = 100, 7, 0.002
    return dict(data=dict(theta_seed=800 + seed, noise_seed=900 + seed, l=lmax, K=K, m=m, sigma_n=sn),
                run=dict(l_min=3, l_max=lmax, K=K, m=m, sigma_n=sn, J=J, J_tilde=100, seed=seed, n_mcmc=5,
                         s_pcn=0.5))


# name -> (data recipe, sampler arguments)
CASES = {
    "batch_J384_l6_s0": _batch_case(384, 6, 0),
    "batch_J512_l6_s1": _batch_case(512, 6, 1),
    "batch_J256_l7_s2": _batch_case(256, 7, 2),
    "stage_benchmark_h8-64_K50_J1000": dict(
        data=dict(theta_seed=4242, noise_seed=4243, l=6, K=50, m=5, sigma_n=0.005),
        run=dict(l_min=3, l_max=6, K=50, m=5, sigma_n=0.005, J=1000, J_tilde=100, seed=11, n_mcmc=5, s_pcn=0.5)),
}


def data_of(d):
    """the synthetic data y of a case (oracle forward map plus seeded noise)"""
    th = inputs.theta_batch(d["theta_seed"], 1, d["K"])
    G = oracle.forward(d["l"], d["K"], 1.0, 0.3, d["m"], th)[0]
    return G + d["sigma_n"] * inputs.rng(d["noise_seed"]).standard_normal(d["m"] * d["m"])


def run_case(c):
    r = oracle.run_sampler(data_of(c["data"]), **c["run"])
    th = r["theta"]
    return dict(n_stages=int(r["n_stages"]), final_level=int(r["final_level"]), final_beta=float(r["final_beta"]),
                stage_type=r["stage_type"].tolist(), stage_level=r["stage_level"].tolist(),
                stage_beta=r["stage_beta"].tolist(), stage_zeta=r["stage_zeta"].tolist(),
                stage_acc_rate=r["stage_acc_rate"].tolist(), solves=[int(v) for v in r["solves"]],
                accepted=int(r["accepted"]), log_Z=float(r["log_Z"]), theta_mean=th.mean(0).tolist(),
                theta_var=th.var(0).tolist())


def main():
    rec = {}
    for name, c in CASES.items():
        rec[name] = dict(case=c, result=run_case(c))
        print(name, rec[name]["result"]["n_stages"], "stages", flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=None, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
