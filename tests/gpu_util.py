"""Helpers for the GPU parity tests (device handling and error measures)."""
import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """max-norm error relative to the max-norm of the reference"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def case(msg):
    print(f"[case] {msg}", flush=True)


def stored_oracle_run(name, data, run):
    """An oracle sampler run stored in tests/golden/oracle_runs.json (written
    by tests/golden/make_oracle_runs.py from oracle/ alone).  The caller
    states the case it expects; a stored case with other data or sampler
    arguments is an error, so a stale file cannot pass silently."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_runs.json")
    rec = json.load(open(path))[name]
    if rec["case"]["data"] != data or rec["case"]["run"] != run:
        raise AssertionError(f"stored oracle run {name} was made for another case; rerun make_oracle_runs.py")
    r = dict(rec["result"])
    for k in ("stage_type", "stage_level"):
        r[k] = np.asarray(r[k], dtype=np.int32)
    for k in ("stage_beta", "stage_zeta", "stage_acc_rate", "theta_mean", "theta_var"):
        r[k] = np.asarray(r[k], dtype=np.float64)
    return r
