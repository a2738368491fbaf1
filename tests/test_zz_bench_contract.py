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


def test_measured_traffic_is_null_once_source_or_shape_differ(tmp_path):
    """`traffic` on the line must come from counters of the same solver
    source and launch shape: a summary with another source hash, or a
    lookup with another shape or form, yields None."""
    good = tmp_path / "good.md"
    good.write_text(f"solver_source_sha256_16: {bench.solver_sha()}\nlaunch_shape: 256,1024,1,0\n"
                    "traffic_bytes_per_launch: 123456789\nlaunch_shape_mixed: 512,512,1,0\n"
                    "traffic_bytes_per_launch_mixed: 987654321\n")
    assert bench.measured_traffic(str(good), (256, 1024, 1, 0)) == 123456789.0
    assert bench.measured_traffic(str(good), (512, 512, 1, 0), "mixed") == 987654321.0
    assert bench.measured_traffic(str(good), (512, 1024, 1, 0)) is None
    assert bench.measured_traffic(str(good), (256, 1024, 1, 0), "mixed") is None
    stale = tmp_path / "stale.md"
    stale.write_text(good.read_text().replace(bench.solver_sha(), "0000000000000000"))
    assert bench.measured_traffic(str(stale), (256, 1024, 1, 0)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), (256, 1024, 1, 0)) is None


def test_byte_models_per_unknown_and_iteration():
    """The streaming models the roofline divides by: FP64 forward without its
    iterate 277 B at V(1,1), the mixed form half of 293 B, each further
    smoothing step 106.7 B (halved for mixed)."""
    assert bench.b_iter(1) == pytest.approx(277.0)
    assert bench.b_iter(2) - bench.b_iter(1) == pytest.approx(106.7)
    assert bench.b_iter(1, True) == pytest.approx(146.5)
    assert bench.b_iter(2, True) - bench.b_iter(1, True) == pytest.approx(53.35)
    # per solve: kappa read, fine and coarse weights written, observations
    n, nobs = 64, 25
    assert bench.solve_bytes(6, nobs, 1, 0, 0) == pytest.approx(8 * 2 * n * n + (4 / 3) * 2 * 2 * n * (n - 1) * 8
                                                              + 32 * nobs)
