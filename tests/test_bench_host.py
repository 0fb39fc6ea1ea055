"""Host-side checks of the benchmark script: its command-line contract on one
GPU, the algorithmic byte and flop model behind `roofline`, and the rule that
stored byte counters are reported only for the kernel sources they were taken
on.  No GPU is touched."""
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
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_link_bytes(bench):
    # SU(2) as a quaternion, SU(3) full and two-row, SU(4); FP32 and FP64
    assert bench.link_bytes(2, "f32") == 16 and bench.link_bytes(2, "f64") == 32
    assert bench.link_bytes(3, "f32") == 72 and bench.link_bytes(3, "f64") == 144
    assert bench.link_bytes(3, "f32r12") == 48 and bench.link_bytes(3, "f64r12") == 96
    assert bench.link_bytes(4, "f32") == 128


def test_phase_and_step_bytes(bench):
    V = 32 ** 4
    # a phase reads the whole field (4V links = 8 x V/2) and writes V/2 links
    assert bench.phase_bytes(3, V, "f32r12") == 9 * 48 * (V // 2) == 226_492_416
    assert bench.phase_bytes(3, V, "f32") == 9 * 72 * (V // 2)
    # 8 phases per update step; re-unitarization reads and writes 4V links,
    # the plaquette reads 4V, the Polyakov loop V
    lb = 72
    assert bench.step_bytes(3, V, "f32", 1, 4) == 40 * 9 * lb * (V // 2) + 13 * V * lb


def test_wide_update_flops(bench):
    # 12 staple products and W = U A at 8 Nc^3 flops each, and two rows of U
    # and W times a 2x2 complex matrix per subgroup
    for nc in (4, 5, 16, 32):
        s = nc * (nc - 1) // 2
        assert bench.wide_update_flops(nc) == 13 * 8 * nc ** 3 + s * 2 * 32 * nc


def test_roofline_fields(bench):
    from paper_1112_4533_amd.workloads import SU3_32_F32_TWO_ROW as run
    r = {"kernels": {"overrelax": {"avg_ms": 0.05, "launches": 10}}}
    line = bench.roofline(run, r)
    assert line["bound"] == "hbm" and line["unit"] == "GB/s" and line["peak"] == 8000.0
    assert line["bytes_per_launch"] == bench.phase_bytes(3, run.volume, run.dtype)
    assert line["achieved"] == pytest.approx(line["bytes_per_launch"] / 0.05e-3 / 1e9)
    assert line["frac"] == pytest.approx(line["achieved"] / 8000.0)
    json.dumps(line)


def test_stored_traffic_follows_the_kernel_sources(bench, tmp_path, monkeypatch):
    entry = {"source_hash": bench.kernel_source_hash(), "read_bytes": 100, "write_bytes": 20}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"w": entry}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic("w") == 120
    assert bench.stored_traffic("other") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)   # the kernels changed
    assert bench.stored_traffic("w") is None


def test_cpu_baseline_fields(bench):
    # the oracle leg on a tiny lattice: the same fields as the 32^4 sample
    from paper_1112_4533_amd.workloads import Run
    run = Run("su3_4^4_hot_f32", 3, (4, 4, 4, 4), 6.2, True, "f32", 1, 4, 1)
    cb = bench.run_cpu_baseline(run, 1)
    assert cb["kind"] == "oracle" and cb["unit"] == "link_updates/s"
    assert cb["value"] > 0 and cb["cores"] >= 1
    assert "1 sweeps" in cb["sample"] and f"{5 * 4 * 4 ** 4} link updates" in cb["sample"]
    json.dumps(cb)
