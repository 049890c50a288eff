"""Throughput benchmark of the TENO5-LAD Euler solver on one MI355X.

Headline workload: 3D periodic compressible turbulence on [0, 2 pi]^3 at
256^3, FP64, gamma = 1.4, rho = 1, p = 1/(gamma Mt^2) with Mt = 0.6,
solenoidal random-phase velocity (E(k) ~ k^4 exp(-2 k^2 / k0^2), k0 = 4,
u_rms = 1, seed 0), CFL 0.5, SSP-RK3 steps through teno_step (the whole hot
path: LF speeds and dt, ghost synthesis, characteristic TENO5-LAD faces along
x, y, z, fused RK stage update), inputs resident in HBM.

metric: cell-updates/s, one cell through one RHS evaluation and its RK stage
update (an RK3 step = 3 cell-updates per cell).

Beside the headline the same JSON line carries
  roofline      the dominant kernel (the slowest sweep) timed with HIP events
                around its launches inside the timed region;
  cpu_baseline  the FP64 oracle timed on the host cores on one RK3 step of
                the same input, and in the same run the GPU's first step
                and one RHS (with every cutoff decision) compared with the
                oracle's over the whole 256^3 field;
  schemes       2D four-quadrant Riemann problem at 2048^2 (eq 4.14 states),
                TENO5-LAD against fixed-cutoff TENO5, TENO5-A (eq 2.16-2.18)
                and the linear upwind scheme, next to the per-step times of
                Table 2;
  table2        the 2D workloads of Table 2 (Rayleigh-Taylor, the two 2D
                Riemann problems, the double Mach reflection) per scheme,
                next to the paper's CPU seconds per step;
  batched       4096 ragged 1D shock tubes (N log-uniform in [128, 4096]),
                500 steps of the persistent graph-replayed batch kernel
                against teno_step per tube on the same GPU;
  adjoint       N = 2048 shock/entropy-wave case, 400 steps: gradient of the
                final density mismatch through the discrete adjoint, against
                the forward run and central finite differences.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras]
       python bench.py --copy-calibration          (plain 1 GiB copies)
       python bench.py --summarize-counters DIR    (rocprofv3 CSV -> profiles/)
       python bench.py --summarize-clock DIR       (GRBM clock counters -> profiles/)
Prints one JSON line (the benchmark modes).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0
METRIC = "TENO RHS cell-updates/s (256³ FP64), % HBM roofline; batched/adjoint vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_3d_256_traffic.txt")
CLOCK_FILE = os.path.join(ROOT, "profiles", "k_sweep_3d_256_clock.txt")
# MI355X: 8 XCDs, whose GRBM_GUI_ACTIVE counts (GPU clock cycles while busy)
# rocprofv3 sums per dispatch; the clock the published FP64 peak assumes
N_XCD = 8
PEAK_CLOCK_GHZ = 2.4
SWEEP_SOURCES = ["paper_2003_09145_amd/csrc/teno_kernels.hip",
                 "paper_2003_09145_amd/csrc/teno_face.hpp",
                 "paper_2003_09145_amd/csrc/teno_device.hpp",
                 "paper_2003_09145_amd/csrc/teno_host.hpp",
                 "paper_2003_09145_amd/csrc/teno_index.hpp",
                 "paper_2003_09145_amd/csrc/teno_divmagic.hpp", "include/teno.h"]
COPY_BYTES = 1 << 30


# --------------------------------------------------------------------------
# Algorithmic operation counts of the literal method (each +, -, *, /, sqrt
# counts 1, an FMA 2; comparisons, max, floor and table lookups count 0;
# a sub-expression shared by several formulas counts once).
# --------------------------------------------------------------------------
def face_flops(nd: int) -> int:
    nc = nd + 2
    roe = 12 + 6 * nd                                # Roe average, b1, b2, c
    left = 12 + 2 * (nd - 1)                         # non-trivial entries of L
    project = 10 * (3 * (2 * nc - 1) + 2 * (nd - 1))  # l.U, l.F, v+-, 6 cells
    recon = 2 * nc * 89                              # eq 2.4-2.15 + LAD, per scalar
    back = nc + 8 * nd + 8                           # f+ + f-, R (f+ + f-)
    return roe + left + project + recon + back


def cell_flops(nd: int) -> int:
    return (9 * nd + 18) + 3 * (nd + 2)  # per-cell staging + flux difference


def rk_flops(nd: int) -> float:
    return (2 + 5 + 5) / 3.0 * (nd + 2)  # eq 4.1-4.3 averaged over the stages


def sweep_flops(nd: int, n, axis: int, fused_rk: bool = False) -> float:
    ncell = math.prod(n[:nd])
    faces = ncell // n[axis] * (n[axis] + 1)
    f = faces * face_flops(nd) + ncell * cell_flops(nd)
    return f + (ncell * rk_flops(nd) if fused_rk else 0.0)


# The same method tallied in its literal evaluation order, per 3D face: the
# characteristic projection of U and F separately and then the split (about
# 486 flop), ten scalar reconstructions with every intermediate of eq 2.8-2.15
# and the LAD cutoff (about 96 each), and the Roe average, eigenvectors,
# back-projection and flux difference (about 125).  This is the per-unit
# figure the roofline's `achieved` uses; the itemized count above is that of
# the operation order the kernels implement.
LITERAL_FACE_FLOPS_3D = 1570


def sweep_flops_literal(n, axis: int, fused_rk: bool = False) -> float:
    ncell = math.prod(n[:3])
    faces = ncell // n[axis] * (n[axis] + 1)
    return faces * LITERAL_FACE_FLOPS_3D + (ncell * rk_flops(3) if fused_rk else 0.0)


def sweep_bytes(nd: int, n, axis: int, fused_rk: bool = False) -> float:
    """Algorithmic HBM bytes of one sweep launch: read U, read the partial RHS
    of earlier axes, write the RHS; the last axis also reads u^n in stages 2
    and 3 and writes the stage state instead of the RHS (FP64)."""
    ncell = math.prod(n[:nd])
    nc = nd + 2
    arrays = 2 + (1 if axis > 0 else 0) + ((2.0 / 3.0) if fused_rk else 0.0)
    return 8 * nc * ncell * arrays


def step_bytes_min(nd: int, ncell: int) -> float:
    """Least HBM bytes of one RK3 step of any implementation: each stage
    reads its input state (and u^n in stages 2, 3) and writes its output."""
    return 8 * (nd + 2) * ncell * (2 + 3 + 3)


def sources_sha() -> str:
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# waves per block of the fixed-stride sweeps on a 256^3 grid: x four waves on
# consecutive chunks of one line, y four neighbouring columns, z eight
SWEEP_WAVES = {0: 4, 1: 4, 2: 8}


def match_kernel(names, kernel: str):
    """The entries of `names` that are `kernel` or an instantiation that
    extends its template arguments (k_sweep<3,2,8,false> matches
    k_sweep<3,2,8,false,74,false>)."""
    return [k for k in names if k == kernel or k.startswith(kernel.rstrip(">") + ",")]


def _load_counter_rows(prefix: str, kernel: str, path: str = None):
    """The key=value fields of a committed counter summary's `prefix` line
    for `kernel` (the traffic summary unless `path` names another), or None
    when the sweep sources changed since it was taken."""
    path = TRAFFIC_FILE if path is None else path
    if not os.path.exists(path):
        return None
    sha, vals = None, {}
    for line in open(path):
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith(prefix + " "):
            name, rest = line[len(prefix) + 1:].split(":", 1)
            kv = dict(x.strip().split("=") for x in rest.split(","))
            vals[name.strip()] = kv
    names = match_kernel(vals, kernel)
    if sha != sources_sha() or len(names) != 1:
        return None
    return vals[names[0]]


def load_traffic(kernel: str):
    """Counter-measured HBM bytes per launch of `kernel` from the committed
    summary, or None when the sweep sources changed since it was taken."""
    kv = _load_counter_rows("kernel", kernel)
    return None if kv is None else float(kv["fetch_bytes"]) + float(kv["write_bytes"])


def load_clock_ghz(kernel: str):
    """Mean GPU clock during launches of `kernel` (GRBM_GUI_ACTIVE per XCD
    over the dispatch duration) from the committed summary, or None."""
    kv = _load_counter_rows("clock", kernel, CLOCK_FILE)
    return None if kv is None else float(kv["clock_GHz"])


def load_executed_flop(kernel: str):
    """Executed FP64 flop per launch of `kernel` (SQ_INSTS_VALU_{ADD,MUL,
    TRANS}_F64 + 2 x FMA, x 64 lanes) from the committed summary, or None."""
    kv = _load_counter_rows("valu", kernel)
    return None if kv is None else float(kv["executed_f64_flop"])


# --------------------------------------------------------------------------
# Headline: 3D 256^3 turbulence
# --------------------------------------------------------------------------
def headline(args, B, W, torch):
    t0 = time.time()
    prob, U = W.turbulence_3d(args.n, seed=0)
    print(f"[bench] input {args.n}^3 built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    S = B.Solver(prob, device=dev)
    Ud = torch.from_numpy(U).to(dev)
    S.init(0.0, float("inf"), 0.5)
    for _ in range(args.warmup):
        S.step(Ud)
    stream = torch.cuda.current_stream()
    nev = 2 * 3 * 3
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(args.steps)]
    for row in evs:           # create the events before the timed region
        for e in row:
            e.record(stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        S.step(Ud, events=evs[k])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    ctrl = S.read_ctrl()
    if ctrl.status != 0:
        raise SystemExit(f"non-physical state during the benchmark (status {ctrl.status})")
    ncell = prob.ncell
    value = 3.0 * ncell * args.steps / (ms * 1e-3)
    print(f"[bench] {args.steps} steps in {ms:.1f} ms (wall {wall * 1e3:.1f} ms), t = {ctrl.t:.5f}",
          file=sys.stderr, flush=True)

    # per-launch durations of the sweep kernels of the timed region
    per_axis = []
    for d in range(3):
        durs = [evs[k][2 * (3 * s + d)].elapsed_time(evs[k][2 * (3 * s + d) + 1])
                for k in range(args.steps) for s in range(3)]
        per_axis.append(sum(durs) / len(durs))
    n3 = [args.n] * 3
    dom = max(range(3), key=lambda a: per_axis[a])
    fused = dom == 2
    flops = sweep_flops_literal(n3, dom, fused_rk=fused)
    achieved = flops / (per_axis[dom] * 1e-3) / 1e12
    flops_impl = sweep_flops(3, n3, dom, fused_rk=fused)
    # the plain (digest-free) instantiation; waves per block by axis at 256^3
    kname = f"k_sweep<3,{dom},{SWEEP_WAVES[dom]},false>"
    traffic = load_traffic(kname)
    executed = load_executed_flop(kname)
    clock = load_clock_ghz(kname)
    alg_bytes = sweep_bytes(3, n3, dom, fused_rk=fused)
    roofline = {
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": traffic,
        "kernel": f"{kname} (axis {'xyz'[dom]}{', fused RK stage' if fused else ''})",
        "launch_ms": round(per_axis[dom], 4),
        "flops_per_launch": flops,
        "flops_per_face": LITERAL_FACE_FLOPS_3D,
        # the same launch counted in the implemented operation order
        "flops_per_launch_implemented_order": flops_impl,
        "frac_implemented_order": round(flops_impl / (per_axis[dom] * 1e-3) / 1e12 /
                                        PEAK_FP64_TFLOPS, 4),
        "algorithmic_bytes_per_launch": alg_bytes,
        "hbm_algorithmic_GBs": round(alg_bytes / (per_axis[dom] * 1e-3) / 1e9, 1),
        "hbm_algorithmic_frac": round(alg_bytes / (per_axis[dom] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "hbm_counter_GBs": (None if traffic is None else
                            round(traffic / (per_axis[dom] * 1e-3) / 1e9, 1)),
        # executed FP64 operations from the committed counters (rocprofv3
        # SQ_INSTS_VALU_*_F64 of the same kernel) over the same launch time
        "fp64_counter_flop_per_launch": executed,
        "fp64_counter_frac": (None if executed is None else
                              round(executed / (per_axis[dom] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)),
        # the GPU clock this kernel sustains (committed GRBM counter summary)
        # and the FP64 peak scaled to it: the published peak assumes 2.4 GHz
        "sustained_clock_GHz": clock,
        "peak_at_sustained_clock": (None if clock is None else
                                    round(PEAK_FP64_TFLOPS * clock / PEAK_CLOCK_GHZ, 1)),
        "frac_at_sustained_clock": (None if clock is None else
                                    round(achieved / (PEAK_FP64_TFLOPS * clock / PEAK_CLOCK_GHZ),
                                          4)),
        "sweep_ms_xyz": [round(x, 4) for x in per_axis],
    }
    step_s = ms * 1e-3 / args.steps
    whole = {
        "cell_steps_per_s": ncell * args.steps / (ms * 1e-3),
        "hbm_min_bytes_per_step": step_bytes_min(3, ncell),
        "hbm_min_frac": round(step_bytes_min(3, ncell) / step_s / 1e9 / PEAK_HBM_GBS, 4),
        "fp64_tflops_algorithmic": round(
            3 * sum(sweep_flops_literal(n3, d, fused_rk=(d == 2)) for d in range(3)) / step_s / 1e12, 3),
        "fp64_tflops_implemented_order": round(
            3 * sum(sweep_flops(3, n3, d, fused_rk=(d == 2)) for d in range(3)) / step_s / 1e12, 3),
        "sweeps_share_of_step": round(3 * sum(per_axis) / (ms / args.steps), 4),
    }
    return prob, U, value, ms, roofline, whole


# --------------------------------------------------------------------------
# f1: scheme variants on the 2D four-quadrant Riemann problem at 2048^2
# --------------------------------------------------------------------------
def schemes_leg(args, B, W, torch):
    """Per-RHS time of each scheme on the same state (the linear scheme is
    not stable on this problem, so its steps would stop at once), and per-step
    time of the two stable ones over the configured run."""
    prob0, U = W.riemann_2d(args.n2d)
    Ud0 = torch.from_numpy(U).cuda()
    out = {"workload": f"2D four-quadrant Riemann problem {args.n2d}^2 (eq 4.14 states, split "
                       f"(0.8, 0.8)), transmissive, CFL 0.5, {args.steps2d} steps",
           "paper_table2_2048_s_per_step": {"TENO5": 13.1, "TENO5-A": 17.8, "Present": 13.7,
                                            "hardware": "desktop workstation CPU (Table 2)"}}
    reps = 20
    for name, kw in (("lad", {}), ("teno5_ct1e-5", {"scheme": "fixed_ct", "ct_fixed": 1e-5}),
                     ("teno5a", {"scheme": "teno5a"}), ("linear5", {"scheme": "linear5"})):
        prob = prob0.replace(**kw)
        S = B.Solver(prob)
        R = S.rhs(Ud0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            S.rhs(Ud0, out=R)
        e1.record()
        torch.cuda.synchronize()
        rec = {"rhs_ms": round(e0.elapsed_time(e1) / reps, 4)}
        if name != "linear5":
            Ud = Ud0.clone()
            S.init(0.0, float("inf"), 0.5)
            S.step(Ud)
            Ud = Ud0.clone()
            S.init(0.0, float("inf"), 0.5)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps2d):
                S.step(Ud)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps2d
            c = S.read_ctrl()
            rec.update({"ms_per_step": round(ms, 4),
                        "cell_updates_per_s": 3.0 * prob.ncell / (ms * 1e-3),
                        "status": int(c.status), "t": c.t})
        out[name] = rec
    base = out["teno5_ct1e-5"]
    out["lad_over_teno5_step"] = round(out["lad"]["ms_per_step"] / base["ms_per_step"], 4)
    out["lad_over_teno5_rhs"] = round(out["lad"]["rhs_ms"] / base["rhs_ms"], 4)
    out["linear5_over_teno5_rhs"] = round(out["linear5"]["rhs_ms"] / base["rhs_ms"], 4)
    out["teno5a_over_teno5_step"] = round(out["teno5a"]["ms_per_step"] / base["ms_per_step"], 4)
    out["teno5a_over_teno5_rhs"] = round(out["teno5a"]["rhs_ms"] / base["rhs_ms"], 4)
    print(f"[bench] schemes 2D: step LAD {out['lad']['ms_per_step']:.3f} ms, TENO5 "
          f"{base['ms_per_step']:.3f} ms, TENO5-A {out['teno5a']['ms_per_step']:.3f} ms; "
          f"rhs LAD {out['lad']['rhs_ms']:.3f}, TENO5 "
          f"{base['rhs_ms']:.3f}, linear {out['linear5']['rhs_ms']:.3f} ms",
          file=sys.stderr, flush=True)
    return out


# --------------------------------------------------------------------------
# f3: the 2D workloads of Table 2, each scheme timed on the same GPU
# --------------------------------------------------------------------------
TABLE2 = [  # case, grid, builder, paper seconds per step (WENO-Z, TENO5, TENO5-A, Present)
    ("Rayleigh-Taylor", "128x512", lambda W: W.rayleigh_taylor(128, 512), (0.14, 0.15, 0.2, 0.16)),
    ("Rayleigh-Taylor", "256x1024", lambda W: W.rayleigh_taylor(256, 1024), (0.59, 0.67, 0.88, 0.70)),
    ("2D Riemann case 1 (eq 4.14)", "1024x1024", lambda W: W.riemann_2d_table2(1, 1024),
     (2.57, 2.89, 3.71, 2.99)),
    ("2D Riemann case 2 (eq 4.13)", "1024x1024", lambda W: W.riemann_2d_table2(2, 1024),
     (2.56, 2.85, 3.68, 2.99)),
    ("2D Riemann case 2 (eq 4.13)", "2048x2048", lambda W: W.riemann_2d_table2(2, 2048),
     (11.9, 13.1, 17.8, 13.7)),
    ("Double Mach reflection", "1024x256", lambda W: W.double_mach(1024, 256),
     (0.59, 0.66, 0.87, 0.69)),
]


def t_final_of(case):
    """Final times of the Sec. 4.3 runs."""
    if case.startswith("Rayleigh"):
        return 1.95
    if case.startswith("2D Riemann case 1"):
        return 0.3
    if case.startswith("2D Riemann case 2"):
        return 0.25
    if case.startswith("Double"):
        return 0.2
    return None


def sod_leg(args, B, W, torch):
    """The Sod shock tube (N = 200, CFL 0.5, to t = 0.2): the whole run as
    teno_step calls and as replays of a recorded graph of steps
    (teno_runner), wall time of each and whether the end states agree bit
    for bit.  On a grid this small every kernel is short, so launch cost
    decides the time."""
    prob, U = W.sod(200)
    out = {"workload": "1D Sod shock tube N=200 on [0, 1], transmissive, CFL 0.5, to t = 0.2"}
    ends = {}
    for mode in ("steps", "graph", "steps", "graph"):   # second pass timed
        S = B.Solver(prob)
        u = torch.from_numpy(U.copy()).cuda()
        S.init(0.0, 0.2, 0.5)
        if mode == "graph":
            S.run(u, 10, steps_per_graph=10)   # records the graph (untimed)
            S.init(0.0, 0.2, 0.5)
            u.copy_(torch.from_numpy(U))
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        if mode == "graph":
            S.run(u, 200, steps_per_graph=10)
        else:
            for _ in range(200):
                S.step(u)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        c = S.read_ctrl()
        ends[mode] = u.cpu()
        out[mode] = {"wall_ms": round(wall * 1e3, 3), "steps": int(c.nsteps), "t": c.t,
                     "status": int(c.status), "enqueued_steps": 200}
    out["graph_over_steps_speedup"] = round(out["steps"]["wall_ms"] / out["graph"]["wall_ms"], 2)
    out["bitwise_equal"] = bool(torch.equal(ends["steps"], ends["graph"]))
    print(f"[bench] sod200 to t=0.2: steps {out['steps']['wall_ms']} ms, graph "
          f"{out['graph']['wall_ms']} ms ({out['steps']['steps']} steps), bitwise "
          f"{out['bitwise_equal']}", file=sys.stderr, flush=True)
    return out


def table2_leg(args, B, W, torch):
    """Per-step time of TENO5-LAD, TENO5 and TENO5-A on the Table 2 workloads
    (timed from the initial condition), with the parameter adjustments the
    paper states: TENO5-A alpha_2 = 5.5, C_r = 0.3 for Riemann case 1 and the
    double Mach reflection, TENO5 C_T = 1e-5 for the double Mach reflection;
    TENO5 C_T = 1e-7 otherwise (Sec. 4)."""
    rows = []
    for case, grid_s, build, paper in TABLE2:
        prob0, U = build(W)
        Ud0 = torch.from_numpy(U).cuda()
        dmr = case.startswith("Double")
        adjust_a = case.startswith("2D Riemann case 1") or dmr
        schemes = {
            "lad": {},
            "teno5": {"scheme": "fixed_ct", "ct_fixed": 1e-5 if dmr else 1e-7},
            "teno5a": dict({"scheme": "teno5a"}, **({"a2": 5.5, "cr": 0.3} if adjust_a else {})),
        }
        row = {"case": case, "grid": grid_s,
               "paper_s_per_step": dict(zip(("WENO-Z", "TENO5", "TENO5-A", "Present"), paper))}
        for name, kw in schemes.items():
            prob = prob0.replace(**kw)
            S = B.Solver(prob)
            Ud = Ud0.clone()
            S.init(0.0, float("inf"), 0.5)
            S.step(Ud)
            Ud = Ud0.clone()
            S.init(0.0, float("inf"), 0.5)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.table2_steps):
                S.step(Ud)
            e1.record()
            torch.cuda.synchronize()
            c = S.read_ctrl()
            ok = c.status == 0 and c.nsteps == args.table2_steps
            # steps after a non-physical state are no-ops: no valid timing then
            row[name] = {"ms_per_step": (round(e0.elapsed_time(e1) / args.table2_steps, 4)
                                         if ok else None),
                         "status": int(c.status), "steps_done": int(c.nsteps)}
        base = row["teno5"]["ms_per_step"]
        row["ratio_to_teno5"] = {k: (round(row[k]["ms_per_step"] / base, 3)
                                     if row[k]["ms_per_step"] and base else None)
                                 for k in ("lad", "teno5", "teno5a")}
        row["paper_ratio_to_teno5"] = {"lad": round(paper[3] / paper[1], 3),
                                       "teno5a": round(paper[2] / paper[1], 3)}
        if row["lad"]["ms_per_step"]:
            row["speedup_vs_paper_present"] = round(paper[3] * 1e3 / row["lad"]["ms_per_step"], 1)
        if t_final_of(case) is not None and grid_s in ("128x512", "1024x1024", "1024x256"):
            # TENO5-LAD with the paper's parameters to the paper's final time
            # (the double Mach reflection also with H = 1, and with H = 10
            # under the cut form of the eq 3.2 sensor: theta = 0 where max
            # chi-tilde > H)
            runs = {"lad_full_run": {}}
            if case.startswith("Double"):
                runs["lad_H1_full_run"] = {"H": 1.0}
                runs["lad_cut_full_run"] = {"theta": "cut"}
            for key, kw in runs.items():
                S = B.Solver(prob0.replace(**kw))
                Ud = Ud0.clone()
                S.init(0.0, t_final_of(case), 0.5)
                w0 = time.perf_counter()
                for k in range(100000):
                    S.step(Ud)
                    if k % 200 == 199:
                        c = S.read_ctrl()
                        if c.status != 0 or not c.t < t_final_of(case):
                            break
                c = S.read_ctrl()
                row[key] = {"t_end": t_final_of(case), "t": c.t, "steps": int(c.nsteps),
                            "status": int(c.status), "rho_min": float(Ud[0].min()),
                            "wall_s": round(time.perf_counter() - w0, 3)}
        rows.append(row)
        fmt = lambda v: "n/a" if v is None else f"{v:.3f}"
        print(f"[bench] table 2 {case} {grid_s}: LAD {fmt(row['lad']['ms_per_step'])} ms, "
              f"TENO5 {fmt(base)} ms, TENO5-A {fmt(row['teno5a']['ms_per_step'])} ms",
              file=sys.stderr, flush=True)
    return {"steps": args.table2_steps, "cases": rows}


# --------------------------------------------------------------------------
# a12: batched ragged 1D tubes against teno_step per tube
# --------------------------------------------------------------------------
def batched_leg(args, B, W, torch):
    import numpy as np
    import tempfile
    batch = W.batched_tubes()
    total = int(batch.offsets[-1])
    cache = os.path.join(tempfile.mkdtemp(prefix="teno_tune_"), "batch_tune.jsonl")
    P = B.BatchPlan(batch.lengths, batch.dx, tune_cache=cache)
    U0 = torch.from_numpy(batch.U.copy()).cuda()
    t0 = time.perf_counter()
    Ud = U0.clone()
    tune_ms = P.autotune(Ud, steps=3)
    tune_s = time.perf_counter() - t0
    waves, bpc = P.config()
    # warm-up (builds the graph), then the timed run from the initial state
    Ud = U0.clone()
    P.init(Ud)
    P.run(Ud, 10)
    Ud = U0.clone()
    P.init(Ud)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    P.run(Ud, args.batch_steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    t, dt, st, ns = P.read()
    # a tube whose state turns non-physical is frozen at its last good step
    # (status 3, as the oracle run of that tube does); it counts the steps it made
    frozen = np.nonzero(st != 0)[0]
    if np.any(st[frozen] != 3) or np.any(ns[st == 0] != args.batch_steps) or len(frozen) > 8:
        raise SystemExit(f"batched run: unexpected tube states (status {np.unique(st)})")
    done = float(np.sum(batch.lengths * ns))
    rate = 3.0 * done / (ms * 1e-3)

    # the plain solver: teno_step per tube, one stream, tubes one after another
    solvers, tubes = [], []
    for b in range(batch.nbatch):
        S = B.Solver(batch.tube_problem(b))
        S.init(0.0, float("inf"), 0.5)
        solvers.append(S)
        o0, o1 = int(batch.offsets[b]), int(batch.offsets[b + 1])
        tubes.append(U0[:, o0:o1].clone().reshape(3, 1, 1, o1 - o0))
    solvers[0].step(tubes[0].clone())  # load / warm the kernels once
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.plain_steps):
        for S, u in zip(solvers, tubes):
            S.step(u)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - w0
    plain_rate = 3.0 * total * args.plain_steps / plain_s
    # same steps through the batch: every tube must match its plain run
    Ub = U0.clone()
    P.init(Ub)
    for _ in range(args.plain_steps):
        P.step(Ub)
    torch.cuda.synchronize()
    plain = torch.cat([u.reshape(3, -1) for u in tubes], dim=1)
    diff = float((plain - Ub).abs().max())
    print(f"[bench] batched: {ms:.1f} ms for {args.batch_steps} steps ({rate:.3e} cell-updates/s); "
          f"plain {plain_rate:.3e}; max |diff| {diff}", file=sys.stderr, flush=True)
    return {
        "workload": f"{batch.nbatch} Sod-type tubes, N log-uniform in [128, 4096] (sum {total}), "
                    f"seeded states, transmissive, CFL 0.5, per-tube dt",
        "steps": args.batch_steps, "ms": round(ms, 3),
        "cell_updates_per_s": rate,
        "nonphysical_tubes": [{"tube": int(b), "cells": int(batch.lengths[b]),
                               "steps_done": int(ns[b])} for b in frozen],
        "autotuned": {"waves_per_block": waves, "blocks_per_cu": bpc,
                      "ms_per_step_tuning": round(tune_ms, 4), "tuning_wall_s": round(tune_s, 2)},
        "plain_per_tube": {"steps": args.plain_steps, "wall_s": round(plain_s, 3),
                           "cell_updates_per_s": plain_rate},
        "speedup_vs_plain": round(rate / plain_rate, 2),
        "max_abs_diff_vs_plain": diff,
    }


# --------------------------------------------------------------------------
# a13: discrete adjoint against the forward solver and finite differences
# --------------------------------------------------------------------------
def adjoint_3d_timing(args, B, W, torch, reps=5):
    """teno_rhs and teno_rhs_adjoint on the 3D turbulence field of
    --adjoint-n3d cells per axis (frozen speeds), ms per call (HIP events)."""
    p3, U3 = W.turbulence_3d(args.adjoint_n3d, seed=0)
    S3 = B.Solver(p3)
    U3d = torch.from_numpy(U3).cuda()
    R3 = S3.rhs(U3d)
    a3 = S3.alpha.clone()
    g3 = B.grid(p3)
    ws3 = torch.empty(B.adjoint_workspace_bytes(g3), dtype=torch.uint8, device="cuda")
    lam3 = torch.ones_like(U3d)
    G3 = torch.empty_like(U3d)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(reps):
            fn()
        a1.record()
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    rhs3_ms = timed(lambda: S3.rhs(U3d, alpha_in=a3, out=R3))
    adj3_ms = timed(lambda: B.teno_rhs_adjoint(g3, U3d, a3, lam3, G3, ws3))
    del ws3, G3, lam3, R3, U3d
    return rhs3_ms, adj3_ms


def adjoint_leg(args, B, W, torch):
    import numpy as np
    from paper_2003_09145_amd.adjoint import Recorder
    N, steps = 2048, args.adjoint_steps
    prob, U0 = W.adjoint_case(N, noise=0.01)
    _, Ut = W.adjoint_case(N, noise=0.0)
    dx = prob.dx[0]
    rec = Recorder(prob)
    # kernel-level ratio on the initial state: teno_rhs_adjoint / teno_rhs
    S = rec.S
    Ud = torch.from_numpy(U0.copy()).cuda()
    R = S.rhs(Ud)
    alpha = S.alpha.clone()
    lam = torch.ones_like(Ud)
    G = torch.empty_like(Ud)
    reps = 200

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(reps):
            fn()
        a1.record()
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    rhs_ms = timed(lambda: S.rhs(Ud, alpha_in=alpha, out=R))
    adj_ms = timed(lambda: B.teno_rhs_adjoint(rec.g, Ud, alpha, lam, G, rec.ws_adj))

    # the same ratio on a 3D field (kernel-bound rather than launch-bound)
    rhs3_ms, adj3_ms = adjoint_3d_timing(args, B, W, torch)

    tgt, _, _ = rec.forward(torch.from_numpy(Ut.copy()).cuda(), steps, 0.5)
    rho_star = tgt[0].clone()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    UK, log, ckpt = rec.forward(Ud, steps, 0.5, seg=20, digest=True)
    torch.cuda.synchronize()
    fwd_s = time.perf_counter() - w0
    base_digest = rec.digest()
    lamT = torch.zeros_like(UK)
    lamT[0] = dx * (UK[0] - rho_star)
    w0 = time.perf_counter()
    lam0 = rec.backward(lamT, log, ckpt, seg=20)
    torch.cuda.synchronize()
    bwd_s = time.perf_counter() - w0
    lam0 = lam0.cpu().numpy()
    u0 = U0[1] / U0[0]
    grad_rho = lam0[0] + u0 * lam0[1] + 0.5 * u0 * u0 * lam0[2]

    def J(Uin):
        UT = rec.replay(torch.from_numpy(Uin).cuda(), log, digest=True)
        return 0.5 * dx * float(((UT[0] - rho_star) ** 2).sum()), rec.digest()

    rng = np.random.default_rng(3)
    cand = rng.permutation(np.nonzero(prob.centres(0) >= -4.0)[0])
    h = 1e-6
    # bar: 1e-6 relative where |dJ/drho_i| >= 0.1 max|dJ/drho|, else 1e-7 max|dJ/drho|
    # (the rounding floor of a central difference at h = 1e-6 grows as 1/h)
    gmax = float(np.abs(grad_rho).max())
    errs, ratios, skipped, tried = [], [], 0, 0
    w0 = time.perf_counter()
    for i in cand:
        if len(errs) == args.fd_cells or tried == 4 * args.fd_cells:
            break
        tried += 1
        dU = np.zeros_like(U0)
        dU[0, 0, 0, i] = 1.0
        dU[1, 0, 0, i] = u0[0, 0, i]
        dU[2, 0, 0, i] = 0.5 * u0[0, 0, i] ** 2
        Jp, dp = J(U0 + h * dU)
        Jm, dm = J(U0 - h * dU)
        if dp != base_digest or dm != base_digest:
            skipped += 1
            continue
        fd = (Jp - Jm) / (2 * h)
        ad = float(grad_rho[0, 0, i])
        errs.append(abs(fd - ad) / max(abs(ad), 1e-300))
        ratios.append(abs(fd - ad) / (1e-6 * max(abs(ad), 0.1 * gmax)))
    fd_s = time.perf_counter() - w0
    worst = max(errs) if errs else None
    print(f"[bench] adjoint 3D {args.adjoint_n3d}^3: rhs {rhs3_ms:.3f} ms, rhs_adjoint {adj3_ms:.3f} ms",
          file=sys.stderr, flush=True)
    print(f"[bench] adjoint: rhs {rhs_ms:.4f} ms, rhs_adjoint {adj_ms:.4f} ms; forward {fwd_s:.3f} s, "
          f"backward {bwd_s:.3f} s; FD {len(errs)} cells, max rel {worst}, {skipped} skipped",
          file=sys.stderr, flush=True)
    return {
        "workload": f"1D N={N} on [-5, 5], Mach-3 shock into rho = 1 + 0.2 sin 5x + noise 0.01, "
                    f"{steps} steps, CFL 0.5, checkpoints every 20 steps",
        "rhs_ms": round(rhs_ms, 5), "rhs_adjoint_ms": round(adj_ms, 5),
        "rhs_adjoint_over_rhs": round(adj_ms / rhs_ms, 3),
        "rhs_3d": {"workload": f"3D turbulence {args.adjoint_n3d}^3", "rhs_ms": round(rhs3_ms, 4),
                   "rhs_adjoint_ms": round(adj3_ms, 4),
                   "rhs_adjoint_over_rhs": round(adj3_ms / rhs3_ms, 3)},
        "forward_recorded_s": round(fwd_s, 4), "backward_s": round(bwd_s, 4),
        "gradient_over_forward": round(bwd_s / fwd_s, 3),
        "fd_check": {"h": h, "cells": len(errs), "skipped_mask_change": skipped,
                     "max_rel_err": worst, "grad_inf": gmax,
                     "bar": "|fd - ad| <= 1e-6 max(|ad|, 0.1 max|grad|)",
                     "max_err_over_bar": max(ratios) if ratios else None,
                     "pass": bool(ratios) and max(ratios) <= 1.0, "wall_s": round(fd_s, 2)},
    }


# --------------------------------------------------------------------------
# Measured HBM bandwidth: a plain device copy
# --------------------------------------------------------------------------
def hbm_copy_bandwidth(torch, nbytes=2 << 30, reps=10):
    """GB/s of a plain device-to-device copy of nbytes (read + write counted),
    HIP events over `reps` copies; the arrays far exceed the 256 MB
    memory-side cache."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


# --------------------------------------------------------------------------
# The oracle on the host cores
# --------------------------------------------------------------------------
def cpu_baseline(prob, U, B=None, torch=None):
    """The oracle timed on one RK3 step of the headline input.  With the
    binding given, the same run also checks the GPU against the oracle on
    that input, element by element over the whole field: the first RK3 step
    (both from U) and one RHS evaluation with every cutoff decision, against
    the fused-order oracle and the FMA-free one."""
    import numpy as np
    import oracle
    U0 = np.ascontiguousarray(U)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.time()
    Uc, _, dtc, _, stc = oracle.step(prob, U0, 0.5, 0.0, float("inf"))
    el = time.time() - t0
    out = {"value": 3.0 * prob.ncell / el, "unit": "cell-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"one SSP-RK3 step (3 RHS evaluations + stage updates) of the same "
                     f"{prob.n[0]}^3 input, {el:.1f} s wall on {threads} OpenMP threads"}
    if B is None:
        return out
    nc = prob.nc

    def rel(a, c):
        scale = np.abs(c).reshape(nc, -1).max(axis=1)
        scale = np.where(scale > 0, scale, 1.0)
        return float((np.abs(a - c).reshape(nc, -1).max(axis=1) / scale).max())

    S = B.Solver(prob)
    Ud = torch.from_numpy(U0).cuda()
    S.init(0.0, float("inf"), 0.5)
    S.step(Ud)
    torch.cuda.synchronize()
    Ug = Ud.cpu().numpy()
    par = {"step_max_rel": rel(Ug, Uc), "step_bitwise": bool(np.array_equal(Ug, Uc)),
           "step_dt_equal": S.read_ctrl().dt == dtc}
    del Ug, Uc
    Ud.copy_(torch.from_numpy(U0))
    R, dec = S.rhs(Ud, decisions=True)
    torch.cuda.synchronize()
    Rg, dg = R.cpu().numpy(), dec.cpu().numpy()
    del R, dec, Ud, S
    torch.cuda.empty_cache()
    t1 = time.time()
    Rc, dc = oracle.rhs(prob, U0, dump=True)
    par.update({"rhs_flips": int(np.count_nonzero(dg != dc)), "rhs_max_rel": rel(Rg, Rc),
                "rhs_bitwise": bool(np.array_equal(Rg, Rc))})
    del Rc, dc
    Rl, dl = oracle.rhs(prob, U0, dump=True, literal=True)
    # against the FMA-free oracle the error is measured per component relative
    # to the larger of the component's largest RHS and its largest
    # back-projection term sum_s |R_cs f^_s| / dx: the mass RHS of this nearly
    # solenoidal field is a small residual of much larger cancelling terms
    _, _, fmax = oracle.rhs_flux_abs(prob, U0, literal=True, with_max=True)
    scale = np.maximum(np.abs(Rl).reshape(nc, -1).max(axis=1), fmax)
    par.update({"literal_rhs_flips": int(np.count_nonzero(dg != dl)),
                "literal_rhs_max_rel": float((np.abs(Rg - Rl).reshape(nc, -1).max(axis=1) /
                                              scale).max()),
                "literal_rhs_max_rel_own_norm": rel(Rg, Rl)})
    par["cells_compared"] = prob.ncell
    par["oracle_check_wall_s"] = round(time.time() - t1, 2)
    out["parity"] = par
    print(f"[bench] 256^3 parity: step bitwise {par['step_bitwise']}, rhs flips {par['rhs_flips']} "
          f"bitwise {par['rhs_bitwise']}; literal oracle flips {par['literal_rhs_flips']} "
          f"max rel {par['literal_rhs_max_rel']:.2e}", file=sys.stderr, flush=True)
    return out


# --------------------------------------------------------------------------
# Counter plumbing: a plain copy of known size, and the CSV summariser
# --------------------------------------------------------------------------
def copy_calibration():
    import torch
    n = COPY_BYTES // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 3}))


def _read_counters(d):
    """{kernel name: {counter: (mean value per dispatch, dispatches)}} from the
    rocprofv3 output under directory d (counter_collection CSV files, else the
    counters_collection view of its SQLite databases)."""
    rows = []
    for p in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(p, newline="") as f:
            for r in csv.DictReader(f):
                key = {k.lower(): v for k, v in r.items()}
                rows.append((p + key.get("dispatch_id"), key.get("kernel_name"),
                             key.get("counter_name"), float(key.get("counter_value"))))
    if not rows:
        import sqlite3
        for p in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
            c = sqlite3.connect(p)
            for dsp, k, cn, v in c.execute(
                    "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
                rows.append((p + str(dsp), k, cn, float(v)))
            c.close()
    per = {}
    for dsp, k, cn, v in rows:
        per[(dsp, k, cn)] = per.get((dsp, k, cn), 0.0) + v
    acc = {}
    for (dsp, k, cn), v in per.items():
        acc.setdefault(k, {}).setdefault(cn, []).append(v)
    return {k: {c: (sum(v) / len(v), len(v)) for c, v in cs.items()} for k, cs in acc.items()}


def _short(name):
    import re
    m = re.search(r"(k_\w+)(<[^>]*>)?", name)
    if not m:
        return name[:60]
    return m.group(1) + (m.group(2) or "").replace(" ", "").replace("(int)", "")


def summarize_clock(d):
    """profiles/k_sweep_3d_256_clock.txt from a GRBM_GUI_ACTIVE run under
    d/grbm: per kernel, the busy GPU cycles per dispatch, the dispatch
    duration and their ratio per XCD, the clock the kernel ran at."""
    per = {}
    for p in glob.glob(os.path.join(d, "grbm", "**", "*counter_collection.csv"), recursive=True):
        with open(p, newline="") as f:
            for r in csv.DictReader(f):
                key = {k.lower(): v for k, v in r.items()}
                if key.get("counter_name") != "GRBM_GUI_ACTIVE":
                    continue
                dur = float(key["end_timestamp"]) - float(key["start_timestamp"])
                per.setdefault(_short(key["kernel_name"]), []).append(
                    (float(key["counter_value"]), dur))
    lines = [
        "# GPU clock during the 3D sweeps and the LF-speed reduction, 256^3 turbulence",
        "#",
        "# command (from the repository root, after cd /tmp && export TMPDIR=/tmp; $OUT is any",
        "# output directory):",
        "#   rocprofv3 --pmc GRBM_GUI_ACTIVE GRBM_COUNT --output-format csv -d $OUT/grbm -o g -- "
        "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-extras",
        "#   python3 bench.py --summarize-clock $OUT",
        f"# clock_GHz = GRBM_GUI_ACTIVE / {N_XCD} XCDs / dispatch duration (rocprofv3 sums the",
        "# counter over the XCDs); the published FP64 peak of 78.6 TFLOP/s assumes 2.4 GHz",
        f"source_sha256: {sources_sha()}",
        "#",
    ]
    for k in sorted(per):
        if not (k.startswith("k_sweep<3") or k.startswith("k_alpha<3")):
            continue
        v = per[k]
        cyc = sum(a for a, _ in v) / len(v)
        dur = sum(b for _, b in v) / len(v)
        lines.append(f"clock {k}: grbm_gui_active={cyc:.0f}, duration_ns={dur:.0f}, "
                     f"clock_GHz={cyc / N_XCD / dur:.3f}, dispatches={len(v)}")
    with open(CLOCK_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(d):
    fetch = _read_counters(os.path.join(d, "fetch"))
    write = _read_counters(os.path.join(d, "write"))
    calf = _read_counters(os.path.join(d, "calf"))
    calw = _read_counters(os.path.join(d, "calw"))
    valu = _read_counters(os.path.join(d, "valu"))
    mix = _read_counters(os.path.join(d, "mix")) if os.path.isdir(os.path.join(d, "mix")) else {}

    def copy_kib(tab, counter):
        best = None
        for k, cs in tab.items():
            if counter in cs and ("copy" in k.lower() or "elementwise" in k.lower()):
                v = cs[counter][0]
                best = v if best is None else max(best, v)
        return best

    cf_kib = copy_kib(calf, "FETCH_SIZE")
    cw_kib = copy_kib(calw, "WRITE_SIZE")
    cal_f = COPY_BYTES / (cf_kib * 1024.0)
    cal_w = COPY_BYTES / (cw_kib * 1024.0)
    n3 = [256] * 3
    lines = [
        "# HBM traffic and FP64 VALU counters of the 3D sweep kernels, 256^3 turbulence",
        "# (k_sweep<3,d,W>: axis d, W waves per block; axis z carries the fused RK stage update)",
        "#",
        "# commands (from the repository root, after cd /tmp && export TMPDIR=/tmp; $OUT is any",
        "# output directory):",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/fetch -o fetch -- "
        "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-extras",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/write -o write -- "
        "python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-extras",
        "#   rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 "
        "SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVES "
        "--output-format csv -d $OUT/valu -o valu -- python3 bench.py --steps 5 "
        "--warmup 1 --no-cpu-baseline --no-extras",
        "#   rocprofv3 --pmc SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_CVT "
        "SQ_INSTS_LDS SQ_INSTS_SALU SQ_WAIT_INST_LDS SQ_WAIT_INST_ANY SQ_INSTS_VALU_FLOPS_FP64 "
        "--output-format csv -d $OUT/mix -o mix -- python3 bench.py --steps 5 --warmup 1 "
        "--no-cpu-baseline --no-extras",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/calf -o calf -- "
        "python3 bench.py --copy-calibration",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/calw -o calw -- "
        "python3 bench.py --copy-calibration",
        "#   python3 bench.py --summarize-counters $OUT",
        "#",
        f"# copy calibration: a plain {COPY_BYTES} B device copy reads FETCH_SIZE = {cf_kib:.0f} KiB "
        f"and WRITE_SIZE = {cw_kib:.0f} KiB per dispatch",
        f"calibration_fetch: {cal_f:.4f}",
        f"calibration_write: {cal_w:.4f}",
        f"source_sha256: {sources_sha()}",
        "#",
        "# per dispatch (mean over dispatches): counter KiB, calibrated bytes, algorithmic bytes",
    ]
    for k in sorted(fetch):
        sk = _short(k)
        if not sk.startswith("k_sweep<3"):
            continue
        fk, nd = fetch[k]["FETCH_SIZE"]
        wk = None
        for kk, cs in write.items():
            if _short(kk) == sk and "WRITE_SIZE" in cs:
                wk = cs["WRITE_SIZE"][0]
        axis = int(sk.split(",")[1])
        fb = fk * 1024.0 * cal_f
        wb = (wk or 0.0) * 1024.0 * cal_w
        alg = sweep_bytes(3, n3, axis, fused_rk=(axis == 2))
        lines.append(f"kernel {sk}: fetch_kib={fk:.0f}, write_kib={wk or 0:.0f}, "
                     f"fetch_bytes={fb:.0f}, write_bytes={wb:.0f}, algorithmic_bytes={alg:.0f}, "
                     f"ratio={(fb + wb) / alg:.3f}, dispatches={nd}")
    lines.append("#")
    lines.append("# FP64 VALU instructions per dispatch (wave-level; x64 lanes; FMA = 2 flop)")
    for k in sorted(valu):
        sk = _short(k)
        if not sk.startswith("k_sweep<3"):
            continue
        cs = valu[k]
        g = lambda c: cs.get(c, (0.0, 0))[0]
        flop = 64.0 * (g("SQ_INSTS_VALU_ADD_F64") + g("SQ_INSTS_VALU_MUL_F64") +
                       g("SQ_INSTS_VALU_TRANS_F64") + 2.0 * g("SQ_INSTS_VALU_FMA_F64"))
        axis = int(sk.split(",")[1])
        alg = sweep_flops_literal(n3, axis, fused_rk=(axis == 2))
        impl = sweep_flops(3, n3, axis, fused_rk=(axis == 2))
        lines.append(f"valu {sk}: add_f64={g('SQ_INSTS_VALU_ADD_F64'):.0f}, "
                     f"mul_f64={g('SQ_INSTS_VALU_MUL_F64'):.0f}, "
                     f"fma_f64={g('SQ_INSTS_VALU_FMA_F64'):.0f}, "
                     f"trans_f64={g('SQ_INSTS_VALU_TRANS_F64'):.0f}, "
                     f"valu_all={g('SQ_INSTS_VALU'):.0f}, waves={g('SQ_WAVES'):.0f}, "
                     f"active_inst_valu={g('SQ_ACTIVE_INST_VALU'):.0f}, "
                     f"busy_cycles={g('SQ_BUSY_CYCLES'):.0f}, executed_f64_flop={flop:.4e}, "
                     f"algorithmic_flop={alg:.4e}, implemented_order_flop={impl:.4e}")
    if mix:
        lines.append("#")
        lines.append("# instruction mix per wave (wave-level instruction counts / SQ_WAVES of the valu")
        lines.append("# pass; other VALU = all VALU - FP64 arithmetic - INT32 - INT64 - CVT: compares,")
        lines.append("# selects, moves, exponent/mantissa operations and lane reads/writes)")
        for k in sorted(mix):
            sk = _short(k)
            if not sk.startswith("k_sweep<3"):
                continue
            waves = None
            for kk, cs in valu.items():
                if _short(kk) == sk:
                    waves = cs.get("SQ_WAVES", (0.0, 0))[0]
                    g = lambda c: cs.get(c, (0.0, 0))[0]
                    f64 = (g("SQ_INSTS_VALU_ADD_F64") + g("SQ_INSTS_VALU_MUL_F64") +
                           g("SQ_INSTS_VALU_FMA_F64") + g("SQ_INSTS_VALU_TRANS_F64"))
                    allv = g("SQ_INSTS_VALU")
            if not waves:
                continue
            m = lambda c: mix[k].get(c, (0.0, 0))[0] / waves
            other = allv / waves - f64 / waves - m("SQ_INSTS_VALU_INT32") - m(
                "SQ_INSTS_VALU_INT64") - m("SQ_INSTS_VALU_CVT")
            lines.append(f"mix {sk}: valu={allv / waves:.0f}, fp64={f64 / waves:.0f}, "
                         f"int32={m('SQ_INSTS_VALU_INT32'):.0f}, int64={m('SQ_INSTS_VALU_INT64'):.0f}, "
                         f"cvt={m('SQ_INSTS_VALU_CVT'):.0f}, other_valu={other:.0f}, "
                         f"lds={m('SQ_INSTS_LDS'):.0f}, salu={m('SQ_INSTS_SALU'):.0f}, "
                         f"wait_inst_lds={m('SQ_WAIT_INST_LDS'):.0f}, "
                         f"wait_inst_any={m('SQ_WAIT_INST_ANY'):.0f}")
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


TRACE_FILE = os.path.join(ROOT, "profiles", "k_sweep_3d_256_kernel_trace.txt")


def summarize_trace(d, bench_json=None):
    """profiles/k_sweep_3d_256_kernel_trace.txt from a rocprofv3 --kernel-trace
    --stats run of the headline (DIR/trace/*kernel_stats.csv) and, if given,
    the JSON line of a default bench.py run (its HIP-event sweep averages)."""
    import csv
    import glob
    path = glob.glob(os.path.join(d, "trace", "*kernel_stats.csv"))
    if not path:
        raise SystemExit(f"no kernel_stats.csv under {d}/trace")
    rows = list(csv.DictReader(open(path[0])))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [
        "# rocprofv3 kernel-trace summary: 3D periodic turbulence 256^3, TENO5-LAD, SSP-RK3",
        "#",
        "# command (repository root, after cd /tmp && export TMPDIR=/tmp; $OUT is any output "
        "directory):",
        "#   rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/trace -o trace -- "
        "python3 bench.py --no-cpu-baseline --no-extras",
        "#   python3 bench.py --summarize-trace $OUT [bench.json of a default run]",
        "# (the headline of the default bench.py run: 3 warm-up + 100 timed steps, 3 stages each,",
        "#  so 309 launches of each per-stage kernel)",
        f"source_sha256: {sources_sha()}",
        "#",
        f"{'kernel':58s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
        f"{'share_%':>8s}",
    ]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].replace("void ", "").replace("teno::", "").split("(")[0]
        lines.append(f"{name[:58]:58s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{100.0 * float(r['TotalDurationNs']) / total:8.2f}")
    if bench_json:
        b = json.loads(open(bench_json).read().strip().splitlines()[-1])
        sw = b["roofline"]["sweep_ms_xyz"]
        lines += ["#",
                  "# same kernels timed inside bench.py's timed region with HIP events around each",
                  "# launch (teno_step_timed, default run: 100 steps, inputs resident in HBM):",
                  f"#   sweep x / y / z average launch: {sw[0] * 1e3:.1f} / {sw[1] * 1e3:.1f} / "
                  f"{sw[2] * 1e3:.1f} us; ms per RK3 step {b['ms_per_step']:.3f}"]
    with open(TRACE_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


ADJ_TRACE_FILE = os.path.join(ROOT, "profiles", "k_adj_chunk_3d_128_kernel_trace.txt")


def summarize_adjoint_trace(d, log=None):
    """profiles/k_adj_chunk_3d_128_kernel_trace.txt from a rocprofv3
    --kernel-trace --stats run of `bench.py --adjoint-3d-only`
    (DIR/adj/*kernel_stats.csv) and, if given, that run's JSON line."""
    import csv
    import glob
    path = glob.glob(os.path.join(d, "adj", "*kernel_stats.csv"))
    if not path:
        raise SystemExit(f"no kernel_stats.csv under {d}/adj")
    rows = list(csv.DictReader(open(path[0])))
    lines = [
        "# rocprofv3 kernel-trace summary: discrete adjoint of the RHS against the RHS,",
        "# 3D periodic turbulence 128^3, TENO5-LAD, frozen speeds (teno_rhs_adjoint 6 calls,",
        "# teno_rhs 7; the first timed call of each is a warm-up)",
        "#",
        "# command (repository root, after cd /tmp && export TMPDIR=/tmp; $OUT is any output "
        "directory):",
        "#   rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/adj -o adj -- "
        "python3 bench.py --adjoint-3d-only",
        "#   python3 bench.py --summarize-adjoint-trace $OUT [its JSON line]",
        "# k_adj_chunk: pass A per axis; k_adj_gather: pass B, once for all axes; k_sweep: the",
        "# forward sweeps of teno_rhs",
        f"source_sha256: {sources_sha()}",
        "#",
        f"{'kernel':58s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}",
    ]
    keep = ("k_adj_", "k_sweep", "k_copy_alpha", "k_alpha")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].replace("void ", "").replace("teno::", "").split("(")[0]
        if not name.startswith(keep):
            continue
        lines.append(f"{name[:58]:58s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f}")
    if log:
        # the run's JSON line (the log may also hold the profiler's messages)
        js = [ln for ln in open(log).read().splitlines() if ln.startswith('{"adjoint_3d"')]
        b = json.loads(js[-1])["adjoint_3d"]
        lines += ["#", "# HIP events around 5 calls each in the same run:",
                  f"#   teno_rhs {b['rhs_ms']:.4f} ms, teno_rhs_adjoint {b['rhs_adjoint_ms']:.4f} ms, "
                  f"ratio {b['rhs_adjoint_over_rhs']:.3f}"]
    with open(ADJ_TRACE_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--n2d", type=int, default=2048)
    ap.add_argument("--steps2d", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--table2-steps", type=int, default=10)
    ap.add_argument("--adjoint-n3d", type=int, default=128)
    ap.add_argument("--fd-cells", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only (no schemes / batched / adjoint legs)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--summarize-counters", metavar="DIR")
    ap.add_argument("--summarize-clock", metavar="DIR")
    ap.add_argument("--summarize-trace", nargs="+", metavar=("DIR", "BENCH_JSON"))
    ap.add_argument("--adjoint-3d-only", action="store_true",
                    help="time teno_rhs and teno_rhs_adjoint on the 3D field only (profiling)")
    ap.add_argument("--summarize-adjoint-trace", nargs="+", metavar=("DIR", "JSON"))
    args = ap.parse_args()
    if args.summarize_clock:
        summarize_clock(args.summarize_clock)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace[:2])
        return
    if args.summarize_adjoint_trace:
        summarize_adjoint_trace(*args.summarize_adjoint_trace[:2])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on exactly one GPU (--gpus 1); sharding over several "
              "GPUs is a design note only", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    from paper_2003_09145_amd import binding as B
    from paper_2003_09145_amd import workloads as W

    B.lib()
    if args.adjoint_3d_only:
        r3, a3 = adjoint_3d_timing(args, B, W, torch)
        print(json.dumps({"adjoint_3d": {"workload": f"3D turbulence {args.adjoint_n3d}^3",
                                         "rhs_ms": r3, "rhs_adjoint_ms": a3,
                                         "rhs_adjoint_over_rhs": a3 / r3}}), flush=True)
        return
    prob, U, value, ms, roofline, whole = headline(args, B, W, torch)
    copy_gbs = hbm_copy_bandwidth(torch)
    roofline["hbm_copy_measured_GBs"] = round(copy_gbs, 1)
    roofline["hbm_algorithmic_frac_of_measured"] = round(
        roofline["hbm_algorithmic_GBs"] / copy_gbs, 4)
    print(f"[bench] plain device copy: {copy_gbs:.1f} GB/s", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
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
        "config": {"workload": f"3D periodic Euler turbulence {args.n}^3 on [0, 2pi]^3, Mt=0.6, "
                               f"k0=4, u_rms=1, seed 0; SSP-RK3 CFL 0.5; TENO5-LAD "
                               f"characteristic reconstruction of global-LF split fluxes",
                   "cells": prob.ncell, "parallelism": "single GPU"},
        "roofline": roofline,
        "step": whole,
    }
    if not args.no_extras:
        out["schemes"] = schemes_leg(args, B, W, torch)
        out["sod"] = sod_leg(args, B, W, torch)
        out["table2"] = table2_leg(args, B, W, torch)
        # the batched kernels are held off the GPU while an unexplained GPU
        # fault reported during their parity test has no cause
        out["batched"] = {"skipped": "batched kernels held off the GPU: an unexplained GPU fault "
                                     "was reported during their parity test"}
        out["adjoint"] = adjoint_leg(args, B, W, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, U, B, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
