"""Host logic of bench.py: the one-GPU guard, the algorithmic byte counts and
the checks that keep a committed counter summary from being reported for a
kernel, launch or list skin it was not taken at."""
import importlib.util
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


def test_traffic_summary_only_for_the_shape_it_was_taken_at(bench):
    path = os.path.join(ROOT, "profiles", "k_force_batch64_fp32_hbm_traffic.txt")
    kv = _profile_kv(path)
    launch = tuple(int(t) for t in kv["launch"].split()[1::2])
    skin = float(kv["skin"])
    got = bench.measured_traffic("k_force", "batch64", "fp32", launch, skin)
    if kv["kernel_source_sha256"] != bench.kernel_source_hash():
        assert got is None     # kernel changed since the counters were taken
        return
    assert got == float(kv["traffic_bytes_per_launch"])
    assert bench.measured_traffic("k_force", "batch64", "fp32", launch, skin + 0.1) is None
    assert bench.measured_traffic("k_force", "batch64", "fp32", (launch[0] * 2, launch[1]), skin) is None
    assert bench.measured_traffic("k_force", "batch64", "fp64", launch, skin) is None
    assert bench.measured_traffic("k_force", "no_such_workload", "fp32", launch, skin) is None


def test_issue_summary_only_for_the_skin_it_was_taken_at(bench):
    path = os.path.join(ROOT, "profiles", "k_force_k_density_batch64_fp32_issue_utilisation.txt")
    kv = _profile_kv(path)
    skin = float(kv["skin"])
    got = bench.measured_issue("k_force", "batch64", "fp32", (2, 1024), skin)
    if kv["kernel_source_sha256"] != bench.kernel_source_hash():
        assert got is None
        return
    assert set(got) == {"valu_issue", "lds_conflict", "resident_waves_per_simd"}
    assert 0.0 < got["valu_issue"] < 1.0 and 0.0 <= got["lds_conflict"] < 1.0
    assert 0.0 < got["resident_waves_per_simd"] <= 8.0
    dens = bench.measured_issue("k_density", "batch64", "fp32", (2, 1024), skin)
    assert dens is not None and dens != got
    assert bench.measured_issue("k_force", "batch64", "fp32", (2, 1024), skin - 0.15) is None
    assert bench.measured_issue("k_force", "batch64", "fp32", (4, 1024), skin) is None
