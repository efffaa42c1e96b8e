"""The benchmark's executed-operation counts are the ones its profile summary
records (for the same kernel sources), and the benchmark refuses multi-GPU
runs with a message."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flux_flop_counts_match_profile():
    import bench

    with open(os.path.join(ROOT, "profiles", "flux_executed_flops_tgv256.md")) as f:
        text = f.read()
    sha = re.search(r"sha256 \([^)]*\): `([0-9a-f]{64})`", text).group(1)
    assert bench.FLUX_EXECUTED["sources_sha256"] == sha
    for key in ("fp64_flop_per_gp", "fp32_flop_per_gp"):
        val = float(re.search(rf"\* {key}: ([0-9.]+)", text).group(1))
        assert bench.FLUX_EXECUTED[key] == val, key
    # the per-lane figure is what the table's FP64 rows give (mean of the directions, within 0.01%)
    # (x and z faces in flux4_kernel<d>, y faces in flux4y_kernel)
    rows = re.findall(r"\| `hgks::flux(?:4_kernel<\d>|4y_kernel)` \|[^\n]*\| ([0-9.]+) \| [0-9.]+ \|", text)
    assert len(rows) == 3
    mean = sum(float(r) for r in rows) / 3
    assert abs(mean - bench.FLUX_EXECUTED["fp64_flop_per_gp"]) <= 1e-4 * mean


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
