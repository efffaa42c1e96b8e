#!/usr/bin/env python3
"""Throughput of the HGKS hot path on one MI355X: cell-stage updates/s of the
Taylor-Green vortex at 256^3 (Ma 0.29, Re 1600, Pr 0.72, CFL 0.5), every step
a full S2O4 step (two stages, each: three directions of reconstruction and
flux, then the cell update; CFL time step reduced on the device).

Prints one JSON line.  `roofline` reports the dominant kernel (the flux
kernel: second tangential sweep, Gauss-point BGK flux, face assembly): the
floating-point operations it executes (hardware counters of the same build)
over its duration, measured by HIP events on the library's stream over the
timed region, against the FP64 vector ALU peak (FP32 for the mixed path).
`hbm_roofline` is the metric's HBM figure: the bytes the method must move per
step (120 per cell-stage) over the step time.  `cpu_baseline` times the oracle
(plain FP64 CPU implementation) on a bounded sample of the same workload.
`repeats` lists the FP64 path's ms/step over the timed block and further
blocks of the same number of steps (their median and run-to-run spread).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-stage updates/s, 256^3 TGV: FP64 vs mixed-FP32 at stated error; % HBM roofline"
UNIT = "cell-stage updates/s"

# Floating-point operations the flux kernel executes per Gauss point (one
# lane), from rocprofv3 --pmc SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F64,F32} over
# whole dispatches of the 256^3 TGV: 64 x (ADD + MUL + TRANS + 2 FMA) per wave
# instruction, divided by the lanes the dispatch launched
# (profiles/flux_executed_flops_tgv256.md; tests/test_bench_constants.py keeps
# the two in step).  The roofline credits only the lanes of distinct faces (4
# per face, n^3 faces per direction on the periodic box), so the padded lanes
# of ragged tiles count for nothing.  Valid for the
# kernel sources they were measured on: `flop_counts_current` says whether the
# sources still hash to those.
FLUX_EXECUTED = {
    "sources_sha256": "c9f871e43af83b38794e06aae81882f87da46814f9d4100844b91d553f293832",
    "fp64_flop_per_gp": 3936.0,   # FP64 flux kernels (their FP32 operations: 4-6 per lane)
    "fp32_flop_per_gp": 3652.0,   # FP32 flux kernel of the mixed path (plus 23 FP64 per lane)
}
# Bytes the method must move per cell-stage (FP64 state): stage 1 reads Q^n
# and writes Q* and the S2O4 accumulator, stage 2 reads Q* and the
# accumulator and writes Q^{n+1}: 6 x 40 B per step, 120 B per cell-stage.
ALGORITHMIC_BYTES_PER_CELL_STAGE = 120.0

# HBM traffic of one flux-kernel launch at 256^3 from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, per dispatch), each divided by the ratio the
# same counter reads for a device copy of known size (bench.py
# --copy-calibration).  Valid only for the kernel sources it was measured on:
# `traffic` is reported as null when their hash differs.
# Mean of the three FP64 directions:
TRAFFIC_MEASURED = {
    "n": 256,
    "sources_sha256": "c9f871e43af83b38794e06aae81882f87da46814f9d4100844b91d553f293832",
    "fetch_bytes": 9.4032e+09,
    "write_bytes": 1.3422e+09,
}

# MI355X published peaks
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def kernel_sources_sha256() -> str:
    """sha256 of the kernel sources with comments, trailing blanks and blank
    lines removed (an edit of a comment leaves it unchanged)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("hgks.hip", "hgks_numerics.hpp"):
        with open(os.path.join(ROOT, "paper_2207_01173_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(line.rstrip() for line in text.split("\n") if line.strip()).encode())
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


def fma_ceiling(blocks: int = 4096, iters: int = 4096, reps: int = 3) -> dict:
    """The FP64 FMA rate this GPU sustains now (library probe: 8 independent
    chains of dependent FMAs per lane), best of `reps` runs timed with events
    on the stream the probe runs on."""
    import torch

    from paper_2207_01173_amd import hgks

    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    hgks.hgks_fma_probe(out.data_ptr(), blocks, 16, stream)  # warm
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        hgks.hgks_fma_probe(out.data_ptr(), blocks, iters, stream)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    tflops = 16.0 * iters * blocks * 256 / best / 1e12
    return {"achieved": round(tflops, 2), "unit": "TFLOP/s", "frac_of_peak": round(tflops / PEAK_FP64_VECTOR_TFLOPS, 4),
            "probe": f"{blocks} x 256 threads, 8 independent chains of {iters} FP64 FMAs per thread"}


def ensemble_bench(steps: int, precision: str) -> dict:
    """64 TGV instances, N from {24, 32, 48, 64, 96}, Ma ~ U[0.1, 0.5], Re ~
    U[400, 3000] (seeded): one batched context (persistent tile launches,
    replayed graph, autotuned shapes) against a loop over per-instance
    contexts, both advancing every instance `steps` CFL steps."""
    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    prec = {"fp64": hgks.FP64, "mixed": hgks.MIXED, "fp32": hgks.FP32}[precision]
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
    def instance_loop(stream):
        """Every instance advanced one step at a time in turn; on a created
        stream each hgks_step replays that instance's captured step, on the
        default stream it launches the kernels one by one.  (Whole-code FP32:
        each of these calls also rounds the state into the FP32 working copy
        and writes it back, which the batch does once per call.)"""
        solvers = [hgks.Solver(p, q, precision=prec, stream=stream) for p, q in zip(params, q0)]
        for s in solvers:
            s.step(1, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for s in solvers:
                s.step(1, 0.0)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        for s in solvers:
            s.close()
        return t

    tl = instance_loop(None)
    print(f"# per-instance loop, plain launches: {tl:.3f} s; with graph replays next", file=sys.stderr, flush=True)
    tg = instance_loop(torch.cuda.Stream())
    cs = 2.0 * cells * steps
    return {
        "metric": "cell-stage updates/s, 64-instance TGV ensemble (N in {24..96}, Ma 0.1-0.5, Re 400-3000)",
        "unit": UNIT, "steps": steps, "precision": precision, "instances": len(params), "cells": cells,
        "batched": {"value": cs / tb, "seconds": tb, "launch_shapes": info},
        "per_instance_loop": {"value": cs / tl, "seconds": tl, "launches": "kernel by kernel"},
        "per_instance_loop_graph": {"value": cs / tg, "seconds": tg, "launches": "one captured step per instance"},
        "speedup": tl / tb,
        "speedup_vs_graph_loop": tg / tb,
    }


def small_grid_steps(n: int, steps: int) -> dict:
    """One TGV instance at n^3 (Ma 0.29): ms per step with the kernels
    launched one by one (default stream) and with the captured step replayed
    (a created stream)."""
    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    p = tgv_workload(n)
    q0 = W.tgv_initial(p)
    out = {"metric": f"ms per S2O4 step, TGV {n}^3, FP64: kernel-by-kernel launches vs one HIP-graph replay",
           "n": n, "steps": steps}
    for name, stream in (("plain", None), ("graph", torch.cuda.Stream())):
        s = hgks.Solver(p, q0, stream=stream)
        s.step(3, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, 0.0)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        s.close()
    out["speedup"] = out["plain_ms_per_step"] / out["graph_ms_per_step"]
    return out


def tgv_history(n: int, ma: float, t_end: float, every: int, with_mixed: bool = True) -> dict:
    """TGV at n^3 (Re 1600, Pr 0.72, CFL 0.5) advanced to t_end by the FP64
    and the mixed path in lockstep, the mixed path on the FP64 run's time
    steps so the two are compared at matched steps: E_k and eps_com every
    `every` steps, and the mixed-minus-FP64 state max-norm when t first
    reaches 1, 2, 5 and 10."""
    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    p = W.tgv_params(n, ma=ma, re=1600.0, pr=0.72, cfl=0.5)
    q0 = W.tgv_initial(p)
    s64 = hgks.Solver(p, q0, precision=hgks.FP64)
    smx = hgks.Solver(p, q0, precision=hgks.MIXED) if with_mixed else None
    keys = ("step", "t", "Ek_fp64", "eps_com_fp64", "Ek_mixed", "eps_com_mixed")
    hist = {k: [] for k in keys}
    marks = [m for m in (1.0, 2.0, 5.0, 10.0) if m <= t_end]
    at_marks = []

    def record(step, st64, stmx):
        for k, v in zip(keys, (step, st64["t"], st64["Ek"], st64["eps_com"],
                               stmx["Ek"] if stmx else None, stmx["eps_com"] if stmx else None)):
            hist[k].append(v)

    record(0, s64.stats(), smx.stats() if smx else None)
    step, t = 0, 0.0
    w0 = time.perf_counter()
    while t < t_end:
        s64.step(1, 0.0)
        st64 = s64.stats()
        if st64["nonfinite"] or not (st64["min_p"] > 0):
            print(f"# FP64 state invalid at step {step + 1} (t = {st64['t']:.4f})", file=sys.stderr, flush=True)
            hist["failed_at_step"] = step + 1
            break
        if smx:
            smx.step(1, st64["dt_last"])
        step += 1
        t = st64["t"]
        hit = bool(marks) and t >= marks[0]
        stmx = None
        if step % every == 0 or hit or t >= t_end:
            stmx = smx.stats() if smx else None
            record(step, st64, stmx)
        if hit and not smx:
            marks.pop(0)
        elif hit:
            a, b = s64.q, smx.q
            rel = ((b - a).abs().amax(dim=(1, 2, 3)) / a.abs().amax(dim=(1, 2, 3))).tolist()
            mom = float((b[1:4] - a[1:4]).abs().max() / a[1:4].pow(2).sum(dim=0).sqrt().max())
            at_marks.append({"t_mark": marks.pop(0), "t": t, "step": step, "state_rel_maxnorm": rel,
                             "momentum_rel_to_max_speed": mom,
                             "Ek_rel": abs(stmx["Ek"] - st64["Ek"]) / st64["Ek"],
                             "eps_com_rel": abs(stmx["eps_com"] - st64["eps_com"]) / st64["eps_com"]})
            print(f"# t={t:.4f} step {step}: mixed-fp64 state rel max-norm {rel}", file=sys.stderr, flush=True)
        if step % 500 == 0:
            print(f"# step {step} t={t:.4f} E_k={st64['Ek']:.6e} ({time.perf_counter() - w0:.0f} s)",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    s64.close()
    if smx:
        smx.close()
    return {"metric": f"TGV {n}^3 E_k and eps_com histories, FP64" + (" and mixed at matched steps" if smx else ""),
            "n": n, "ma": ma, "re": 1600.0, "steps": step, "t_end": t, "every": every,
            "wall_s": wall, "mixed_vs_fp64": at_marks, "history": hist}


def channel_run(n: int, t_end: float, every: int, mass_flux: bool = False) -> dict:
    """Turbulent channel (2 pi x 2 x pi, n^3, tanh-stretched y, isothermal
    walls, Ma_b 0.5, Re_b 3000, constant body force, Poiseuille + 10% noise)
    advanced to t_end by the FP64 and the mixed path in lockstep (the mixed
    path on the FP64 run's time steps).  Every `every` steps: wall shear stress
    on both walls and bulk velocity from x-z plane means; at the end the mean
    U(y) and T(y) of both paths and their state max-norm difference."""
    import numpy as np
    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    p = W.channel_params((n, n, n), ma_b=0.5, re_b=3000.0)
    p["mass_flux_control"] = mass_flux
    q0 = W.channel_initial(p, seed=2207)
    y = torch.as_tensor(W.channel_y_centres(p), dtype=torch.float64, device="cuda")
    ylo, yhi = p["lo"][1], p["hi"][1]
    edges = torch.as_tensor(np.concatenate(([ylo], 0.5 * (W.channel_y_centres(p)[1:] + W.channel_y_centres(p)[:-1]),
                                            [yhi])), dtype=torch.float64, device="cuda")
    dy = edges[1:] - edges[:-1]
    mu_w = p["mu_ref"]  # mu at T = T_w
    gm1 = p["gamma"] - 1.0

    def means(q):
        rho = q[0].mean(dim=(0, 2))
        U = (q[1] / q[0]).mean(dim=(0, 2))
        ke = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
        T = (gm1 * (q[4] - ke) / q[0]).mean(dim=(0, 2))
        return rho, U, T

    def wall_shear(U):
        # dU/dy at each wall from the first two cell centres and U = 0 at the wall
        # (one-sided quadratic through the wall point)
        out = []
        for i0, i1, yw in ((0, 1, ylo), (n - 1, n - 2, yhi)):
            d1, d2 = abs(float(y[i0]) - yw), abs(float(y[i1]) - yw)
            u1, u2 = float(U[i0]), float(U[i1])
            out.append(mu_w * (u1 * d2 * d2 - u2 * d1 * d1) / (d1 * d2 * (d2 - d1)))
        return out

    def bulk(q):
        rho_u = q[1].mean(dim=(0, 2))
        rho = q[0].mean(dim=(0, 2))
        return float((rho_u * dy).sum() / (rho * dy).sum())

    s64 = hgks.Solver(p, q0, precision=hgks.FP64)
    smx = hgks.Solver(p, q0, precision=hgks.MIXED)
    hist = {k: [] for k in ("step", "t", "tau_w_fp64", "tau_w_mixed", "U_b_fp64", "U_b_mixed", "force_fp64",
                            "force_mixed")}

    def record(step, t):
        _, U64, _ = means(s64.q)
        _, Umx, _ = means(smx.q)
        for k, v in (("step", step), ("t", t), ("tau_w_fp64", wall_shear(U64)), ("tau_w_mixed", wall_shear(Umx)),
                     ("U_b_fp64", bulk(s64.q)), ("U_b_mixed", bulk(smx.q)),
                     ("force_fp64", s64.stats()["body_force_x"]), ("force_mixed", smx.stats()["body_force_x"])):
            hist[k].append(v)
        print(f"# step {step} t={t:.4f} tau_w fp64 {hist['tau_w_fp64'][-1]} mixed {hist['tau_w_mixed'][-1]} "
              f"U_b {hist['U_b_fp64'][-1]:.6f} {hist['U_b_mixed'][-1]:.6f} ({time.perf_counter() - w0:.0f} s)",
              file=sys.stderr, flush=True)

    w0 = time.perf_counter()
    record(0, 0.0)
    step, t = 0, 0.0
    while t < t_end:
        s64.step(1, 0.0)
        st64 = s64.stats()
        if st64["nonfinite"] or not (st64["min_p"] > 0):
            raise RuntimeError(f"channel FP64 state invalid at step {step}")
        smx.step(1, st64["dt_last"])
        step += 1
        t = st64["t"]
        if step % every == 0 or t >= t_end:
            record(step, t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    rho64, U64, T64 = means(s64.q)
    rhomx, Umx, Tmx = means(smx.q)
    a, b = s64.q, smx.q
    rel = ((b - a).abs().amax(dim=(1, 2, 3)) / a.abs().amax(dim=(1, 2, 3))).tolist()
    stmx = smx.stats()
    from paper_2207_01173_amd.channel import channel_statistics

    stats = {"fp64": channel_statistics(s64.q, p, y), "mixed": channel_statistics(smx.q, p, y)}
    s64.close()
    smx.close()
    return {"statistics": stats, "metric": f"channel {n}^3 (Ma_b 0.5, Re_b 3000, " + ("constant mass flux" if mass_flux else "constant force")
            + "): wall shear and mean profiles, FP64 and mixed",
            "n": n, "steps": step, "t_end": t, "wall_s": wall, "every": every,
            "mixed_nonfinite": stmx["nonfinite"], "mixed_vs_fp64_state_rel_maxnorm": rel,
            "profiles": {"y": y.tolist(), "U_fp64": U64.tolist(), "U_mixed": Umx.tolist(),
                         "T_fp64": T64.tolist(), "T_mixed": Tmx.tolist(),
                         "rho_fp64": rho64.tolist(), "rho_mixed": rhomx.tolist()},
            "history": hist}


def tgv_workload(n: int):
    from paper_2207_01173_amd import workloads as W

    return W.tgv_params(n, ma=0.29, re=1600.0, pr=0.72, cfl=0.5)


def cpu_baseline(n_sample: int = 64, steps: int = 10) -> dict:
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--repeats", type=int, default=5,
                    help="blocks of --steps steps timed on the FP64 path (the first gives value; all give the spread)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "fp32"], default="fp64", help="precision of --ensemble")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed and FP32 runs beside FP64")
    ap.add_argument("--cpu-sample", type=int, default=64, help="grid of the oracle's timed sample")
    ap.add_argument("--cpu-steps", type=int, default=10, help="S2O4 steps of the oracle's timed sample")
    ap.add_argument("--ensemble", action="store_true",
                    help="measure the 64-instance ensemble (batched vs per-instance loop) instead")
    ap.add_argument("--history", type=float, default=0.0, metavar="T_END",
                    help="instead: TGV --n^3 at Ma --ma to t = T_END, FP64 and mixed histories")
    ap.add_argument("--channel", type=float, default=0.0, metavar="T_END",
                    help="instead: channel at --n^3 to t = T_END, FP64 and mixed wall shear and profiles")
    ap.add_argument("--mass-flux", action="store_true", help="--channel with the constant-mass-flux controller")
    ap.add_argument("--ma", type=float, default=0.1, help="Mach number of --history")
    ap.add_argument("--every", type=int, default=10, help="statistics interval of --history (steps)")
    ap.add_argument("--small-grid", type=int, default=0, metavar="N",
                    help="instead: ms per step at N^3, kernel by kernel vs one graph replay")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the slab-decomposition design is described, not built); run with --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2207_01173_amd import hgks
    from paper_2207_01173_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.small_grid:
        print(json.dumps(small_grid_steps(args.small_grid, args.steps)), flush=True)
        return 0
    if args.ensemble:
        print(json.dumps(ensemble_bench(args.steps, args.precision)), flush=True)
        return 0
    if args.channel > 0:
        print(json.dumps(channel_run(args.n, args.channel, args.every, args.mass_flux)), flush=True)
        return 0
    if args.history > 0:
        print(json.dumps(tgv_history(args.n, args.ma, args.history, args.every, not args.no_mixed)), flush=True)
        return 0
    n = args.n
    p = tgv_workload(n)
    print(f"# building TGV {n}^3 initial state", file=sys.stderr, flush=True)
    q0 = W.tgv_initial(p)

    def run(prec_name: str):
        """Warmup, then K timed CFL steps with per-kernel event timing."""
        prec = {"fp64": hgks.FP64, "mixed": hgks.MIXED, "fp32": hgks.FP32}[prec_name]
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
        faces_per_launch = n * n * n  # every axis periodic: n distinct faces along each normal
        launch_s = flux_ms / flux_n / 1e3
        fp64 = prec == hgks.FP64
        flop_per_gp = FLUX_EXECUTED["fp64_flop_per_gp" if fp64 else "fp32_flop_per_gp"]
        achieved = flop_per_gp * 4 * faces_per_launch / launch_s / 1e12
        peak = PEAK_FP64_VECTOR_TFLOPS if fp64 else PEAK_FP32_VECTOR_TFLOPS
        traffic = measured_traffic(n) if fp64 else None
        roofline = {
            "bound": "alu",
            "kernel": "flux_kernel (2nd tangential WENO-Z sweep + Gauss-point BGK flux + face assembly)",
            "achieved": round(achieved, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic,
            "flops": "executed " + ("FP64" if fp64 else "FP32") + " operations per Gauss point from the "
                     "SQ_INSTS_VALU_* counters (FMA = 2), times 4 Gauss points per face",
            "flop_per_gauss_point": flop_per_gp,
            "flop_counts_current": FLUX_EXECUTED["sources_sha256"] == kernel_sources_sha256(),
            "faces_per_launch": faces_per_launch,
            "avg_launch_ms": round(launch_s * 1e3, 4),
            "kernel_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in prof.items()},
        }
        if not fp64:
            # the build excludes packed FP32 instructions: one FP32 operation
            # per lane and cycle, the rate of FP64
            roofline["frac_of_unpacked_fp32_peak"] = round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4)
        if traffic:
            roofline["traffic_GBs"] = round(traffic / launch_s / 1e9, 1)
            roofline["traffic_frac_of_hbm_peak"] = round(traffic / launch_s / 1e9 / PEAK_HBM_GBS, 4)
        elapsed = t1 - t0
        state = solver.state()
        spread = None
        if prec == hgks.FP64 and args.repeats > 1:
            # run-to-run spread: further blocks of K steps after the timed one
            # (the solution keeps advancing; `value` is the first block)
            per_step = [elapsed / args.steps * 1e3]
            for r in range(args.repeats - 1):
                torch.cuda.synchronize()
                r0 = time.perf_counter()
                solver.step(args.steps, 0.0)
                torch.cuda.synchronize()
                per_step.append((time.perf_counter() - r0) / args.steps * 1e3)
                print(f"# {prec_name}: repeat {r + 2} of {args.repeats}: {per_step[-1]:.3f} ms/step",
                      file=sys.stderr, flush=True)
            spread = {"blocks": args.repeats, "ms_per_step": [round(x, 3) for x in per_step],
                      "median_ms_per_step": round(float(statistics.median(per_step)), 3)}
        solver.close()
        return elapsed, roofline, st, state, spread

    elapsed, roofline, st, state64, spread = run("fp64")
    # the FP64 FMA rate the GPU sustains (clock and issue under FP64 load), as
    # the ceiling beside the published peak
    roofline["sustained_fp64_fma"] = fma_ceiling()
    roofline["frac_of_sustained_fma"] = round(roofline["achieved"] / roofline["sustained_fp64_fma"]["achieved"], 4)
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
        # the metric's HBM figure: bytes the method must move per step over the step time
        "hbm_roofline": {
            "bytes_per_cell_stage": ALGORITHMIC_BYTES_PER_CELL_STAGE,
            "achieved": round(ALGORITHMIC_BYTES_PER_CELL_STAGE * value / 1e9, 2),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(ALGORITHMIC_BYTES_PER_CELL_STAGE * value / 1e9 / PEAK_HBM_GBS, 5),
        },
        # the paper's FP64 single-GPU speedups over its 8-core OpenMP CPU code
        # (TGV, Sec. 4.1 Table 3): context only, other hardware and code
        "paper_context": {
            "fp64_speedup_vs_8core_cpu": {"TITAN RTX": "6.0-7.6 (7x)", "Tesla V100": "15.4-16.1 (16x)"},
            "cpu": "Intel i7-9700, 8 cores, OpenMP",
            "v100_256cubed_cell_stage_updates_per_s": 1.79e7,
        },
    }
    if spread:
        out["repeats"] = spread
    if not args.no_mixed:
        dtypes = {"mixed": "f32 reconstruction and flux on deviations from the mean state, f64 state/update/reductions",
                  "fp32": "f32 state, stages and update, f32 reconstruction and flux, f64 face fluxes and reductions"}
        for name in ("mixed", "fp32"):
            m_elapsed, m_roof, m_st, state_m, _ = run(name)
            # stated error of the reduced-precision path against the FP64 path at matched steps
            rel = (abs(state_m - state64).max(axis=(1, 2, 3)) / abs(state64).max(axis=(1, 2, 3)))
            mom = abs(state_m[1:4] - state64[1:4]).max() / ((state64[1:4] ** 2).sum(axis=0) ** 0.5).max()
            out[name] = {
                "value": cell_stages / m_elapsed,
                "ms_per_step": m_elapsed / args.steps * 1e3,
                "speedup_vs_fp64": elapsed / m_elapsed,
                "dtype": dtypes[name],
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
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, args.cpu_steps)
        out["paper_context"]["this_gpu_fp64_vs_oracle_on_host"] = round(value / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
