"""Host logic of bench.py: the one-GPU guard, the algorithmic byte counts and
the checks that keep a committed counter summary from being reported for a
kernel, launch, list skin or run length it was not taken at."""
import glob
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _profile_kv(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv.setdefault(k.strip(), v.strip())
    return kv


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_atom(bench):
    # force: x, v read and written, x0 read (3 doubles each), own F' (fp32), row length, row of int32 ids
    assert bench.force_bytes_per_atom(0, "fp32") == 2 * 24 + 2 * 24 + 24 + 4 + 4
    assert bench.force_bytes_per_atom(100, "fp32") - bench.force_bytes_per_atom(0, "fp32") == 400
    assert bench.force_bytes_per_atom(0, "fp64") == bench.force_bytes_per_atom(0, "fp32") + 4
    # density: x read, row length and row, F' and F written
    assert bench.density_bytes_per_atom(10, "fp32") == 24 + 4 + 40 + 4 + 8
    assert bench.density_bytes_per_atom(10, "fp64") == 24 + 4 + 40 + 8 + 8


def _run_of(kv):
    """The run a summary was taken on: launch (lanes, block, grid), skin,
    timed steps, warm-up steps."""
    launch = tuple(int(t) for t in kv["launch"].split()[1::2])
    return launch, float(kv["skin"]), int(kv["steps"]), int(kv["warmup"])


def _others(launch, skin, steps, warmup):
    """Runs that differ from the given one in one respect each."""
    lanes, block, grid = launch
    return [((lanes * 2, block, grid), skin, steps, warmup), ((lanes, block // 2, grid), skin, steps, warmup),
            ((lanes, block, grid + 256), skin, steps, warmup), (launch, skin + 0.1, steps, warmup),
            (launch, skin, steps + 1, warmup), (launch, skin, steps, warmup + 1)]


def test_traffic_summary_only_for_the_run_it_was_taken_on(bench):
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_force_*_hbm_traffic.txt")))
    assert paths
    runs = [_run_of(_profile_kv(p)) for p in paths]
    for path, run in zip(paths, runs):
        kv = _profile_kv(path)
        got = bench.measured_traffic("k_force", kv["workload"], kv["precision"], *run)
        if kv["kernel_source_sha256"] != bench.kernel_source_hash():
            assert got is None     # kernel changed since the counters were taken
            continue
        assert got == float(kv["traffic_bytes_per_launch"])
        for other in _others(*run):
            if other not in runs:
                assert bench.measured_traffic("k_force", kv["workload"], kv["precision"], *other) is None
        other_prec = "fp64" if kv["precision"] == "fp32" else "fp32"
        assert bench.measured_traffic("k_force", kv["workload"], other_prec, *run) is None
        assert bench.measured_traffic("k_force", "no_such_workload", kv["precision"], *run) is None


def test_issue_summary_only_for_the_run_it_was_taken_on(bench):
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_force_k_density_*_issue_utilisation.txt")))
    assert paths
    runs = [_run_of(_profile_kv(p)) for p in paths]
    for path, run in zip(paths, runs):
        kv = _profile_kv(path)
        got = bench.measured_issue("k_force", kv["workload"], kv["precision"], *run)
        if kv["kernel_source_sha256"] != bench.kernel_source_hash():
            assert got is None
            continue
        assert set(got) == {"valu_issue", "lds_conflict", "resident_waves_per_simd"}
        assert 0.0 < got["valu_issue"] < 1.0 and 0.0 <= got["lds_conflict"] < 1.0
        assert 0.0 < got["resident_waves_per_simd"] <= 8.0
        dens = bench.measured_issue("k_density", kv["workload"], kv["precision"], *run)
        assert dens is not None and dens != got
        for other in _others(*run):
            if other not in runs:
                assert bench.measured_issue("k_force", kv["workload"], kv["precision"], *other) is None


def _fake_run(force_ms, force_n, steps=20):
    return {"natoms": 113090, "n_rep": 64, "steps": steps, "warmup": 5, "ms": 1.6, "wall_s": 0.002,
            "kt": {"density": (0.0, 0), "force": (force_ms, force_n), "lists": (0.0, 0)},
            "stride": 10, "mean_nl": 70.0, "passes": steps, "rebuilt_reps": 3, "rebuilt_atoms": 5000,
            "end_nl": 71.0, "max_nl": 80, "cap": 160, "launch": (2, 1024, 0), "tuned": (2, 1024, 0.08),
            "desc": "64 replicas", "list_builder": "global"}


class _Args:
    warmup, precision, workload, skin = 5, "fp32", "batch64", 0.65


def test_timing_stride_samples_every_short_run(bench):
    # the driver's short run (20 timed steps) and the default long run both get samples;
    # the first timed iteration is always sampled, so any steps >= 1 has one
    # at most one sample in ten iterations (each event pair costs ~5 us of a 60-80 us step)
    assert bench.timing_stride(1) == 10 and bench.timing_stride(20) == 10
    assert bench.timing_stride(42000) == 50


def test_result_line_with_the_driver_step_counts(bench):
    out = bench.result_line(_Args, _fake_run(0.066, 2), None, None)
    assert out["steps"] == 20 and out["warmup"] == 5
    assert out["config"]["list_builder"] == "global"
    assert out["ms_per_step"] == pytest.approx(1.6 / 20)
    assert out["value"] == pytest.approx(113090 * 20 / 1.6e-3)
    rf = out["roofline"]
    assert rf["avg_launch_us"] == pytest.approx(33.0)
    bpa = bench.force_bytes_per_atom(70.0, "fp32")
    assert rf["achieved"] == pytest.approx(bpa * 113090 / 33e-6 / 1e9)
    assert rf["frac"] == pytest.approx(rf["achieved"] / 8000.0)
    json.dumps(out)


def test_result_line_without_timed_launches_has_no_roofline(bench):
    # timing switched off (or nothing sampled): no division, roofline null
    out = bench.result_line(_Args, _fake_run(0.0, 0), None, None)
    assert out["roofline"] is None
    assert out["value"] > 0
    json.dumps(out)


def test_cpu_baseline_reports_threads_model_and_both_legs(bench):
    cpu = bench.cpu_baseline(target_s=0.3)
    assert cpu["kind"] == "oracle" and cpu["unit"] == "atom-steps/s"
    assert 1 <= cpu["cores"] <= bench.CPU_THREADS_MAX
    assert cpu["value"] > 0 and cpu["single_core"]["value"] > 0 and cpu["single_core"]["cores"] == 1
    assert cpu["host"]["threads_available"] >= 1 and isinstance(cpu["host"]["model"], str)


def test_config_records_and_graph_ratio(bench):
    run = _fake_run(0.066, 2)
    rec = bench.config_record("batch64_fp32_graph", run, "fp32", "batch64", 0.65, 64)
    assert rec["force_roofline_frac"] is None and rec["graph_iterations"] == 64   # no kernel events in a graph
    rec = bench.config_record("rs_scan_fp32", run, "fp32", "rs_scan", 0.65, 0)
    assert rec["force_roofline_frac"] > 0 and rec["value"] == pytest.approx(113090 * 20 / 1.6e-3)
    names = [c[0] for c in bench.CONFIGS]
    assert "batch64_fp32_graph" in names and "batch64_fp32_eager" in names
    out = bench.result_line(_Args, run, None, None, {"x": rec})
    assert out["other_configs"]["x"]["workload"].startswith("rs_scan_fp32")
    json.dumps(out)


def test_free_energy_summary(bench):
    d64 = [-4.0, -4.1, -3.9, -4.2]
    off = [1e-4, -2e-4, 3e-4, 0.0]          # eV/atom
    r = bench.free_energy_summary([a + b for a, b in zip(d64, off)], d64, [100.0, 200.0, 300.0, 400.0],
                                  "four replicas", (5, 20, 5), 1.0)
    import numpy as np
    d = np.array(off) * 1e3
    assert r["mean_meV_per_atom"] == pytest.approx(d.mean(), abs=1e-9)
    assert r["se_meV_per_atom"] == pytest.approx(d.std(ddof=1) / 2.0, abs=1e-9)
    assert r["max_abs_meV_per_atom"] == pytest.approx(0.3, abs=1e-9) and r["T_at_max_K"] == 300.0
    assert r["replicas"] == 4 and r["within_gate"]
    assert "5 steps at lambda 0, 20 forward" in r["protocol"]
    far = bench.free_energy_summary([a + 6e-4 for a in d64], d64, [100.0] * 4, "w", (5, 20, 5), 1.0)
    assert not far["within_gate"] and far["mean_meV_per_atom"] == pytest.approx(0.6, abs=1e-9)
    with pytest.raises(ValueError):
        bench.free_energy_summary([], [], [], "w", (5, 20, 5), 1.0)
    with pytest.raises(ValueError):
        bench.free_energy_summary([float("nan")], [0.0], [100.0], "w", (5, 20, 5), 1.0)
