"""Throughput benchmark of the TENO5-LAD Euler solver on one MI355X.

Workload: 3D periodic compressible turbulence on [0, 2 pi]^3 at 256^3, FP64,
gamma = 1.4, rho = 1, p = 1/(gamma Mt^2) with Mt = 0.6, solenoidal random-phase
velocity (E(k) ~ k^4 exp(-2 k^2 / k0^2), k0 = 4, u_rms = 1, seed 0), CFL 0.5,
SSP-RK3 steps through teno_step (the whole hot path: LF speeds and dt,
ghost synthesis, characteristic TENO5-LAD faces along x, y, z, fused RK
stage update).

metric: cell-updates/s, one cell through one RHS evaluation and its RK stage
update (an RK3 step = 3 cell-updates per cell), inputs resident in HBM.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU (vector)
PEAK_HBM_GBS = 8000.0


# --------------------------------------------------------------------------
# Algorithmic operation counts of the literal method (each +, -, *, /, sqrt
# counts 1; comparisons and table lookups count 0; repeated identical
# sub-expressions count once).  Derivation in the design doc.
# --------------------------------------------------------------------------
def face_flops(nd: int) -> int:
    nc = nd + 2
    roe = 12 + 6 * nd
    left = 12 + 2 * (nd - 1)
    project = 10 * (3 * (2 * nc - 1) + 2 * (nd - 1))
    recon = 2 * nc * 89
    back = nc + 8 * nd + 8
    return roe + left + project + recon + back


def cell_flops(nd: int) -> int:
    return (9 * nd + 18) + 3 * (nd + 2)  # per-cell staging + flux difference


def sweep_flops(nd: int, n, axis: int) -> int:
    ncell = math.prod(n[:nd])
    faces = ncell // n[axis] * (n[axis] + 1)
    return faces * face_flops(nd) + ncell * cell_flops(nd)


def sweep_bytes(nd: int, n, axis: int) -> int:
    """Algorithmic HBM bytes of one sweep: read U, read the partial RHS of
    earlier axes (if any), write the RHS (FP64)."""
    ncell = math.prod(n[:nd])
    nc = nd + 2
    return 8 * nc * ncell * (2 + (1 if axis > 0 else 0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU (--gpus 1); multi-GPU sharding is "
              "design-only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2003_09145_amd import binding as B
    from paper_2003_09145_amd import workloads as W

    t0 = time.time()
    prob, U = W.turbulence_3d(args.n, seed=0)
    print(f"[bench] input {args.n}^3 built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    S = B.Solver(prob, device=dev)
    Ud = torch.from_numpy(U).to(dev)
    S.init(0.0, float("inf"), 0.5)
    for _ in range(args.warmup):
        S.step(Ud)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        S.step(Ud)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ctrl = S.read_ctrl()
    if ctrl.status != 0:
        raise SystemExit(f"non-physical state during the benchmark (status {ctrl.status})")
    ncell = prob.ncell
    value = 3.0 * ncell * args.steps / (ms * 1e-3)
    print(f"[bench] {args.steps} steps in {ms:.1f} ms, t = {ctrl.t:.5f}", file=sys.stderr, flush=True)

    # ---- the dominant kernel: one sweep launch per axis, timed with events on
    # the stream it is launched on ------------------------------------------
    R = torch.empty_like(Ud)
    alpha = torch.tensor([ctrl.alpha[0][0], ctrl.alpha[0][1], ctrl.alpha[0][2]],
                         dtype=torch.float64, device=dev)
    per_axis = []
    for axis in range(3):
        B.teno_sweep(S.g, axis, Ud, R, alpha, Rin=(R if axis else None))
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(args.kernel_reps):
            B.teno_sweep(S.g, axis, Ud, R, alpha, Rin=(R if axis else None))
        a1.record(stream)
        torch.cuda.synchronize()
        per_axis.append(a0.elapsed_time(a1) / args.kernel_reps)
    n3 = [args.n] * 3
    dom = max(range(3), key=lambda a: per_axis[a])
    flops = sweep_flops(3, n3, dom)
    achieved = flops / (per_axis[dom] * 1e-3) / 1e12
    roofline = {
        "bound": "alu",
        "kernel": f"k_sweep<3,{dom},4> (axis {'xyz'[dom]})",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": None,
        "launch_ms": round(per_axis[dom], 4),
        "flops_per_launch": flops,
        "sweep_ms_xyz": [round(x, 4) for x in per_axis],
        "hbm_algorithmic_GBs": round(sweep_bytes(3, n3, dom) / (per_axis[dom] * 1e-3) / 1e9, 1),
    }

    out = {
        "metric": "TENO RHS cell-updates/s (256^3 FP64)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D periodic Euler turbulence {args.n}^3, Mt=0.6, k0=4, "
                               f"SSP-RK3 CFL 0.5, TENO5-LAD characteristic, global LF",
                   "cells": ncell, "parallelism": "single GPU"},
        "roofline": roofline,
    }

    if not args.no_cpu_baseline:
        import oracle
        U0 = np.ascontiguousarray(U)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.time()
        oracle.step(prob, U0, 0.5, 0.0, float("inf"))
        el = time.time() - t0
        out["cpu_baseline"] = {
            "value": 3.0 * ncell / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one SSP-RK3 step (3 RHS + stage updates) of the same {args.n}^3 input, "
                      f"{el:.1f} s wall on {threads} OpenMP threads"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
