#!/usr/bin/env python3
"""Throughput of the HGKS hot path on one MI355X: cell-stage updates/s of the
Taylor-Green vortex at 256^3 (Ma 0.29, Re 1600, Pr 0.72, CFL 0.5), every step
a full S2O4 step (two stages, each: three directions of reconstruction and
flux, then the cell update; CFL time step reduced on the device).

Prints one JSON line.  `roofline` reports the dominant kernel (the flux
kernel: second tangential sweep, Gauss-point BGK flux, face assembly) against
the FP64 vector ALU peak, with its duration measured by HIP events on the
library's stream over the timed region.  `cpu_baseline` times the oracle
(plain FP64 CPU implementation) on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-stage updates/s, 256^3 TGV: FP64 vs mixed-FP32 at stated error; % HBM roofline"
UNIT = "cell-stage updates/s"

# Floating-point operations of the method per face, counted once (no halo
# recomputation) by the oracle's counting scalar (oracle.count_flops(); kept in
# step with it by tests/test_bench_constants.py): second tangential sweep plus
# Gauss-point flux for 4 Gauss points, plus the face assembly, with the moments
# evaluated economically (u separated from v, w, xi; the plain expansion of
# every moment would count 66491).  Every add, multiply, divide, square root
# and transcendental counts as one operation.
FLOPS_FLUX_PER_FACE = 30875.0
# normal sweep plus first tangential sweep (2 Gauss lines) per face
FLOPS_RECON_PER_FACE = 6630.0

# HBM traffic of one flux-kernel launch at 256^3 from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, per dispatch), each divided by the ratio the
# same counter reads for a device copy of known size (bench.py
# --copy-calibration).  Valid only for the kernel sources it was measured on:
# `traffic` is reported as null when their hash differs.
# Mean of the three FP64 directions:
TRAFFIC_MEASURED = {
    "n": 256,
    "sources_sha256": "abdd776e3a8893f200d16cef01f073fc28975dbf580448dc6987feaeb24c5f51",
    "fetch_bytes": 1.2606e+10,
    "write_bytes": 1.4365e+09,
}

# MI355X published peaks
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def kernel_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("hgks.hip", "hgks_numerics.hpp"):
        with open(os.path.join(ROOT, "paper_2207_01173_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n: int):
    if TRAFFIC_MEASURED is None or n != TRAFFIC_MEASURED.get("n", 256):
        return None
    if TRAFFIC_MEASURED["sources_sha256"] != kernel_sources_sha256():
        return None
    return TRAFFIC_MEASURED["fetch_bytes"] + TRAFFIC_MEASURED["write_bytes"]


def copy_calibration(mib: int) -> int:
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (profile this run with rocprofv3 --pmc)."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)
    return 0


def ensemble_bench(steps: int, precision: str) -> dict:
    """64 TGV instances, N from {24, 32, 48, 64, 96}, Ma ~ U[0.1, 0.5], Re ~
    U[400, 3000] (seeded): one batched context (persistent tile launches,
    replayed graph, autotuned shapes) against a loop over per-instance
    contexts, both advancing every instance `steps` CFL steps."""
    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    prec = hgks.FP64 if precision == "fp64" else hgks.MIXED
    params = W.tgv_ensemble(64)
    q0 = [W.tgv_initial(p) for p in params]
    cells = sum(p["n"][0] * p["n"][1] * p["n"][2] for p in params)
    print(f"# ensemble: {len(params)} instances, {cells} cells", file=sys.stderr, flush=True)
    b = hgks.Batch(params, q0, precision=prec)
    info = b.info()
    b.step(1)
    b.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.synchronize()
    tb = time.perf_counter() - t0
    b.close()
    print(f"# batched: {tb:.3f} s; per-instance loop next", file=sys.stderr, flush=True)
    solvers = [hgks.Solver(p, q, precision=prec) for p, q in zip(params, q0)]
    for s in solvers:
        s.step(1, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s in solvers:
            s.step(1, 0.0)
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    for s in solvers:
        s.close()
    cs = 2.0 * cells * steps
    return {
        "metric": "cell-stage updates/s, 64-instance TGV ensemble (N in {24..96}, Ma 0.1-0.5, Re 400-3000)",
        "unit": UNIT, "steps": steps, "precision": precision, "instances": len(params), "cells": cells,
        "batched": {"value": cs / tb, "seconds": tb, "launch_shapes": info},
        "per_instance_loop": {"value": cs / tl, "seconds": tl},
        "speedup": tl / tb,
    }


def tgv_workload(n: int):
    from paper_2207_01173_amd import workloads as W

    return W.tgv_params(n, ma=0.29, re=1600.0, pr=0.72, cfl=0.5)


def cpu_baseline(n_sample: int = 64, steps: int = 1) -> dict:
    """The oracle, as it stands, on the host cores: S2O4 steps of a TGV of the
    same physics at a smaller grid (the per-cell work does not depend on the
    grid size)."""
    from oracle import oracle as O
    from paper_2207_01173_amd import workloads as W

    p = tgv_workload(n_sample)
    q = W.tgv_initial(p)
    O.lib()
    t0 = time.perf_counter()
    O.step(p, q, steps, 0.0)
    t1 = time.perf_counter()
    cs = 2.0 * n_sample ** 3 * steps
    return {
        "value": cs / (t1 - t0),
        "unit": UNIT,
        "cores": O.get_threads(),
        "kind": "oracle",
        "sample": f"{steps} S2O4 step(s) of the {n_sample}^3 TGV (Ma 0.29, Re 1600, Pr 0.72, CFL 0.5), "
                  f"{cs:.0f} cell-stages in {t1 - t0:.2f} s",
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64", help="precision of --ensemble")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision run beside FP64")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--ensemble", action="store_true",
                    help="measure the 64-instance ensemble (batched vs per-instance loop) instead")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the slab-decomposition design is described, not built); run with --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.ensemble:
        print(json.dumps(ensemble_bench(args.steps, args.precision)), flush=True)
        return 0
    n = args.n
    p = tgv_workload(n)
    print(f"# building TGV {n}^3 initial state", file=sys.stderr, flush=True)
    q0 = W.tgv_initial(p)

    def run(prec_name: str):
        """Warmup, then K timed CFL steps with per-kernel event timing."""
        prec = hgks.FP64 if prec_name == "fp64" else hgks.MIXED
        solver = hgks.Solver(p, q0, precision=prec)
        print(f"# {prec_name}: warmup {args.warmup} steps", file=sys.stderr, flush=True)
        solver.step(args.warmup, 0.0)
        torch.cuda.synchronize()
        hgks.hgks_profile(solver.ctx, True)
        hgks.hgks_profile_read(solver.ctx)  # clear
        print(f"# {prec_name}: timing {args.steps} steps", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.step(args.steps, 0.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = hgks.hgks_profile_read(solver.ctx)
        hgks.hgks_profile(solver.ctx, False)
        st = solver.stats()
        if st["nonfinite"] or not (st["min_p"] > 0):
            raise RuntimeError(f"{prec_name}: state became invalid during the benchmark")
        flux_ms, flux_n = prof["flux"]
        faces_per_launch = (n + 1) * n * n
        achieved = FLOPS_FLUX_PER_FACE * faces_per_launch / (flux_ms / flux_n / 1e3) / 1e12
        peak = PEAK_FP64_VECTOR_TFLOPS if prec == hgks.FP64 else PEAK_FP32_VECTOR_TFLOPS
        roofline = {
            "bound": "alu",
            "kernel": "flux_kernel (2nd tangential WENO-Z sweep + Gauss-point BGK flux + face assembly)",
            "achieved": round(achieved, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(n) if prec == hgks.FP64 else None,
            "avg_launch_ms": round(flux_ms / flux_n, 4),
            "flops_per_face": FLOPS_FLUX_PER_FACE,
            "faces_per_launch": faces_per_launch,
            "kernel_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in prof.items()},
        }
        elapsed = t1 - t0
        state = solver.state()
        solver.close()
        return elapsed, roofline, st, state

    elapsed, roofline, st, state64 = run("fp64")
    cell_stages = 2.0 * n ** 3 * args.steps
    value = cell_stages / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"Taylor-Green vortex {n}^3 periodic on [0,2pi]^3, Ma 0.29, Re 1600, Pr 0.72, "
                        f"CFL 0.5 (CFL time step each step)",
            "n": n,
            "precision": "fp64",
            "parallelism": "single GPU",
            "simulated_time": st["t"],
        },
        "roofline": roofline,
    }
    if not args.no_mixed:
        m_elapsed, m_roof, m_st, state_m = run("mixed")
        # stated error of the mixed path against the FP64 path at matched steps
        rel = (abs(state_m - state64).max(axis=(1, 2, 3)) / abs(state64).max(axis=(1, 2, 3)))
        mom = abs(state_m[1:4] - state64[1:4]).max() / ((state64[1:4] ** 2).sum(axis=0) ** 0.5).max()
        out["mixed"] = {
            "value": cell_stages / m_elapsed,
            "ms_per_step": m_elapsed / args.steps * 1e3,
            "speedup_vs_fp64": elapsed / m_elapsed,
            "dtype": "f32 reconstruction and flux on deviations from the mean state, f64 state/update/reductions",
            "error_vs_fp64": {
                "after_steps": args.warmup + args.steps,
                "state_rel_maxnorm": [float(x) for x in rel],
                "momentum_rel_to_max_speed": float(mom),
                "Ek_rel": abs(m_st["Ek"] - st["Ek"]) / st["Ek"],
                "eps_com_rel": abs(m_st["eps_com"] - st["eps_com"]) / st["eps_com"],
            },
            "roofline": m_roof,
        }
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
