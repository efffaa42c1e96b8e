"""The benchmark's per-face operation counts match the oracle's counter, and
the benchmark refuses multi-GPU runs with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flop_constants_match_oracle(oracle):
    import bench

    c = oracle.count_flops()
    flux = 4 * (c["tangential_2_per_gp"] + c["flux_per_gp_lean"]) + c["face_assembly"]
    recon = c["normal_sweep_per_face"] + 2 * c["tangential_1_per_face_gp_line"]
    assert bench.FLOPS_FLUX_PER_FACE == flux
    assert bench.FLOPS_RECON_PER_FACE == recon


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
