"""Host-side checks of bench.py's bookkeeping (no GPU): the algorithmic work
counts it divides by, the kernel it names for each workload, the traffic
profile reader, and the refusal of more than one GPU."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_pass_work_counts_by_hand():
    # 3-way, ranks (2, 3, 4), 10 nonzeros, nonempty slices R = (5, 6, 7); a
    # record is N dwords per nonzero (N - 1 row offsets and the value); the
    # stored slice rows are design bytes, not algorithmic ones
    dims, ranks, nnz, R = (8, 9, 10), (2, 3, 4), 10, (5, 6, 7)
    w = bench.pass_work(dims, ranks, nnz, R, su=4)
    PK = 24
    for n in range(3):
        P = PK // ranks[n]
        flops = 2 * nnz * P + 2 * R[n] * PK
        others = [m for m in range(3) if m != n]
        byts = nnz * 12 + 8 * R[n] + sum(R[m] * ranks[m] * 4 for m in others) + 4 * dims[n] * ranks[n]
        assert w[n] == (flops, byts, 4 * R[n] * P)
    # 16-bit factor copies halve only the factor-row term
    w2 = bench.pass_work(dims, ranks, nnz, R, su=2)
    for n in range(3):
        others = [m for m in range(3) if m != n]
        assert w[n][1] - w2[n][1] == sum(R[m] * ranks[m] * 2 for m in others)


def test_default_workload_is_the_bf16_comparison():
    cfg = bench.CONFIGS["c3"]
    assert cfg["prec"] == "bf16" and cfg["compare"] == "fp32" and cfg["ranks"] == (32, 32, 32)
    assert cfg["nnz"] == 50_000_000 and cfg["dims"] == (1_000_000, 500_000, 20_000)
    assert bench.CONFIGS["c4"]["compare"] == "fp32"


def test_kernel_names_follow_the_library_choice():
    assert bench.ttm_kernel_name((10, 10, 10), (32, 32, 32), "bf16").startswith("k_ttm22<bf16>")
    assert bench.ttm_kernel_name((10, 10, 10), (32, 32, 32), "fp32").startswith("k_ttm<fp32>")
    assert bench.ttm_kernel_name((10,) * 4, (10,) * 4, "fp16").startswith("k_ttm4c<fp16>")
    assert bench.ttm_kernel_name((10,) * 4, (10,) * 4, "fp32").startswith("k_ttm4c<fp32>")
    assert bench.ttm_kernel_name((10,) * 4, (20, 10, 10, 10), "fp16").startswith("k_ttm<fp16>")
    assert bench.ttm_kernel_name((10, 10, 10), (16, 16, 16), "bf16").startswith("k_ttm<bf16>")
    assert bench.ttm_kernel_name((80,) * 5, (10,) * 5, "fp32").startswith("k_gen_rows")


def test_traffic_reader(tmp_path, monkeypatch):
    import hashlib
    h = hashlib.sha256()
    for src in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    good = tmp_path / "good.txt"
    good.write_text(f"# comment: x\nkernel_source_sha256: {h.hexdigest()}\ntraffic_bytes_per_launch: 1234\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_source_sha256: 00\ntraffic_bytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {("g", "fp32"): "good.txt", ("s", "fp32"): "stale.txt"})
    monkeypatch.setattr(bench, "KERNEL_SOURCES", tuple(os.path.join(ROOT, s) for s in bench.KERNEL_SOURCES))
    assert bench.measured_traffic("g", "fp32") == 1234
    assert bench.measured_traffic("s", "fp32") is None  # kernels changed since the counters were taken
    assert bench.measured_traffic("none", "fp32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("config", ["c4", "c3f32", "c1"])
def test_gather_only_refuses_rows_other_than_64_bytes(config):
    # the gather-only pass reads 64-byte rows of 3-way workloads (c2 at 16
    # float32, c3 at 32 bfloat16); other workloads are refused before any
    # device work
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", config, "--gather-only"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "64 bytes" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
