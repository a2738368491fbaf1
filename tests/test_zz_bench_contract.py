"""The benchmark's command-line contract: one GPU only, and one JSON line
with the metric, the roofline of the dominant kernel and the CPU baseline."""
import json
import sys

import pytest

import bench


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_flow_solver_byte_model_counts_the_fused_passes():
    # V(1,1): 48 + 48 + 138 (fine level, FP32 V-cycle weights) + 170 / 3
    # (coarse levels, FP64) B per unknown and iteration, nothing else when
    # the per-solve terms are left out (particles = 0)
    l, iters = 6, 10
    M = (2 ** l - 1) * (2 ** l + 1)
    assert bench.flow_solve_bytes(l, 25, 0, iters, 1) == pytest.approx(iters * M * (96 + 138 + 170 / 3))
    assert bench.flow_solve_bytes(l, 25, 0, iters, 2) - bench.flow_solve_bytes(l, 25, 0, iters, 1) == \
        pytest.approx(iters * M * (128 + 160 / 3))
    # from h = 1/128 on the prolongation pass (18 B) becomes 2 B of coarse
    # values read inside the first black sweep
    l = 8
    M = (2 ** l - 1) * (2 ** l + 1)
    assert bench.flow_solve_bytes(l, 49, 0, iters, 1) == pytest.approx(iters * M * (96 + 122 + 170 / 3))


@pytest.mark.gpu
def test_default_line_keeps_the_contract(monkeypatch, capsys):
    from tests.gpu_util import case, device
    device()
    case("bench default line, 2 steps")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "2", "--warmup", "1", "--no-extras", "--no-autotune",
                                      "--quick-cpu"])
    bench.main()
    line = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")][-1]
    d = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["value"] > 0
    assert d["config"]["workload"] and d["data"] == "synthetic" and d["vs_baseline"] is None
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3 and 0 < rf["frac"] < 1.2
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]


def test_committed_shapes_and_counter_summary_match_the_solver_source():
    """The default line takes its solver launch shapes from the committed
    tuned-shape file and its measured HBM bytes from the committed counter
    summary, each only when it was made for the current solver source (and,
    for the bytes, the same launch shape).  A solver edit without a retune
    and a fresh summary would silently fall back to autotuning and a null
    `traffic`; this keeps the committed files in step with the source."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sha = bench.solver_sha()
    for name in ("mi355x_h16-512_K200_J8192.json", "mi355x_h8-64_K50_J1000.json"):
        rec = json.load(open(os.path.join(root, "paper_1709_09763_amd", "tuned", name)))
        assert rec["solver_source_sha256_16"] == sha, name
        assert rec["device_key"] == "gfx950:256cu"
    rec = json.load(open(os.path.join(root, "paper_1709_09763_amd", "tuned", "mi355x_h16-512_K200_J8192.json")))
    summary = os.path.join(root, "profiles", "solve_h512_K200_J8192_pmc.md")
    for form in ("fp64", "mixed"):
        sh = rec[form]["9"]
        shape = (sh["grid"], sh["block"], sh["nu"], sh["lds"])
        t = bench.measured_traffic(summary, shape, form)
        assert t is not None and 1e12 < t < 3e12, (form, shape)
    # and the h = 1/64 stage workload's summary for its committed h = 1/64 shape
    rec = json.load(open(os.path.join(root, "paper_1709_09763_amd", "tuned", "mi355x_h8-64_K50_J1000.json")))
    sh = rec["fp64"]["6"]
    t = bench.measured_traffic(os.path.join(root, "profiles", "solve_h64_K50_J1000_pmc.md"),
                               (sh["grid"], sh["block"], sh["nu"], sh["lds"]))
    assert t is not None and 1e9 < t < 3e10
