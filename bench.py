"""Throughput of the WENO-C hyperbolic step on one MI355X.

A step is one full third-order SSP Runge-Kutta step (CFL time step on the
device, three RK stages) of every instance.  Default workload: 256
independent shock-bubble instances (grids n x n, n drawn from 64..512, two or
three phases, 27.2 M cells, seed 0), batched in one context, in the mixed
FP32/FP64 precision, WENO-C + HLL, CFL 0.2: the largest single-GPU
configuration of the benchmark set.  The same line reports, on the same
workload and on the 2048 x 1024 two-phase shock-bubble grid, FP64 and mixed
throughput side by side with the L1 / Linf difference of the mixed states
from the FP64 states after the same timed steps.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME]
                  [--precision fp64|mixed] [--no-compare] [--cpu-seconds S]

Inputs are synthetic and seeded (paper_2608_00746_amd.inputs) and resident in
HBM before the timed region.  The roofline entry reports the RK stage (the
sweep kernels of one stage over every instance) against the HBM roof:
algorithmic bytes per stage (8 n_U bytes per cell read of the stage state,
8 n_U per cell read of the step-start state in stages 2 and 3, 8 n_U per cell
written; averaged over the three stages) over the average stage time; the
ALU roof (FP64 flops per stage, FP32 flops at half weight, from the counter
table in profiles/) is nested beside it.  The stage time is measured with
HIP events the library records on its stream around each stage, in a short
eager pass right after the timed steps (those replay a captured graph, whose
events cannot be read back).  `traffic` is the measured HBM bytes per stage
from the counter table, when it holds a row for this workload, tile choice
and kernel source.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 1 FMA (2 flops) x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6
# VALU issue ceiling: one wave64 instruction per SIMD every 4 clocks, i.e.
# 256 x 4 x 16 lane-ops per clock at 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
COUNTER_TABLE = os.path.join(ROOT, "profiles", "stage_counters.md")
WORKLOADS = ["batched_256", "shock_bubble_2048x1024", "shock_interface_n3_1024",
             "advection_2d_512", "advection_1d_200", "shock_vessel_bubble_400x200x200"]


def kernel_source_hash():
    """sha256 over the HIP sources (the counters below hold for this code)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2608_00746_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stage_counters(workload, precision, tiles):
    """Counter figures of one RK stage from the table in profiles/ (rocprofv3
    --pmc runs of this script):

    * traffic: HBM bytes per stage (FETCH_SIZE and WRITE_SIZE runs, scaled by
      a reference copy), only from the row of this workload, precision, tile
      choice and kernel source (else None);
    * flops64, flops32, valu: FP64 and FP32 flops and VALU lane-instructions
      per cell per stage, from the row of this tile choice and kernel source,
      else None."""
    out = {"traffic": None, "flops64": None, "flops32": None, "valu": None}
    if not os.path.exists(COUNTER_TABLE):
        return out
    key = kernel_source_hash()
    for line in open(COUNTER_TABLE):
        cols = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cols) != 9 or cols[0] in ("workload",) or cols[0].startswith("---"):
            continue
        wl, prec, tl, src, fetch_kib, write_kib, f64, f32, valu = cols
        if (wl, prec, src) != (workload, precision, key) or tl != tiles:
            continue
        out.update(flops64=float(f64), flops32=float(f32), valu=float(valu),
                   traffic=(float(fetch_kib) + float(write_kib)) * 1024.0)
    return out


def workload(name, precision):
    """Workloads by name; precision None keeps each workload's own (FP64
    for the advection and shock-bubble problems, mixed for the N = 3
    shock-interface problem and the batched sweep)."""
    from paper_2608_00746_amd import inputs as I
    if name == "advection_2d_512":
        ws = [I.advection_2d(512)]
    elif name == "shock_bubble_2048x1024":
        ws = [I.shock_bubble_2d(2048, 1024)]
    elif name == "shock_interface_n3_1024":
        ws = [I.shock_interface_n3(1024)]
    elif name == "advection_1d_200":
        ws = [I.advection_1d(200)]
    elif name == "batched_256":
        ws = I.batched()
    elif name == "shock_vessel_bubble_400x200x200":
        ws = [I.shock_vessel_bubble_3d(400, 200, 200)]
    else:
        raise SystemExit(f"unknown workload {name}")
    if precision is not None:
        prec = I.PREC_MIXED if precision == "mixed" else I.PREC_FP64
        for w in ws:
            w.opts.precision = prec
    return ws


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(ws, seconds):
    """The oracle as it stands, on the host cores, on a bounded sample: the
    first instance, whole steps until `seconds` have elapsed."""
    from oracle import mpo
    w = ws[0]
    o = w.opts
    pb = mpo.Problem(w.ndim, w.n, w.dx, w.bc, list(w.gamma), list(w.pinf), list(w.D),
                     list(w.pmin), list(w.cT), recon=o.recon, flux=o.flux, model=o.model,
                     energy_limiter=o.energy_limiter, cfl=o.cfl, t_end=0.0,
                     alpha_source=o.alpha_source)
    U = w.U.reshape(-1).copy()
    t0 = time.perf_counter()
    steps = 0
    while True:
        U = pb.step(U, pb.dt(U, 0.0))
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": steps * w.ncells / el, "unit": "cell-updates/s",
            "cores": mpo.num_threads(), "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{steps} full RK3 steps of instance 0 of {len(ws)} "
                      f"({w.name}, {w.ncells} cells, FP64), {el:.1f} s, "
                      f"OpenMP over grid lines"}


def group_order(ws):
    """(d, N) of the library's instance groups, in its group order."""
    return sorted({(w.ndim, w.N) for w in ws})


def tiles_key(args, ws, tiles):
    """The tile choice as x<lanes>/y<X>x<Y>/<plain|xcd>: one entry when every
    group has the same shapes, else one per group (comma-separated, in group
    order), the form --tiles takes."""
    if args.tiles:
        return args.tiles
    if tiles is None:
        return "default"
    per = []
    for g in group_order(ws):
        i = next(k for k, w in enumerate(ws) if (w.ndim, w.N) == g)
        t = tiles[i].tolist()
        per.append("x%d/y%dx%d/%s" % (t[0], t[1], t[2], "xcd" if t[3] else "plain"))
    return per[0] if len(set(per)) == 1 else ",".join(per)


def tiles_env(spec):
    """Environment of the library's tile overrides for a --tiles spec."""
    xl, yl, sl = [], [], []
    for ent in spec.split(","):
        xs, ys, sw = ent.split("/")
        yx, yy = (int(v) for v in ys[1:].split("x"))
        xl.append(str([256, 128, 64].index(int(xs[1:]))))
        # 1D groups report a y tile of 0 x 0: any index serves
        yl.append(str([(16, 16), (32, 8), (16, 24), (0, 0)].index((yx, yy)) % 3))
        sl.append({"plain": "0", "xcd": "1"}[sw])
    return {"MPWENO_XSHAPE": ",".join(xl), "MPWENO_YSHAPE": ",".join(yl),
            "MPWENO_XCD_SWIZZLE": ",".join(sl)}


def measure(ws, args, stream, keep_state=False):
    """One timed run: set-up, autotune, W warm-up steps, capture of the
    16-step graph, K timed steps (events on the solver stream, bracketed by
    device synchronisation), then an eager pass with stage events."""
    import torch
    from paper_2608_00746_amd.binding import Solver
    s = Solver(ws, stream=stream, use_graph=not args.no_graph)
    tiles = None if (args.no_autotune or args.tiles) else s.autotune()
    s.advance(args.warmup)
    s.advance(0)                    # capture the 16-step graph outside the timed region
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.advance(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    d = s.diag()
    if (d[:, 25] > 0).any():
        raise SystemExit("non-finite state after the timed steps")
    state = [s.host(i).copy() for i in range(len(ws))] if keep_state else None
    t_reached = d[:, 26].copy()
    prof_steps = max(1, min(args.steps, 20))
    s.profile(3)
    for _ in range(prof_steps):
        s.step()
    k_ms, k_n = s.timing(reset=True)
    s.profile(0)
    s.close()
    cells = sum(w.ncells for w in ws)
    print("measured %d instance(s), %d cells, precision %d: %.4g cell-updates/s, "
          "%.4g ms/step, stage %.4g ms" % (len(ws), cells, ws[0].opts.precision,
                                           cells * args.steps / (ms / 1e3), ms / args.steps,
                                           k_ms / max(k_n, 1)), file=sys.stderr, flush=True)
    return {"value": cells * args.steps / (ms / 1e3), "ms_per_step": ms / args.steps,
            "wall_s": wall, "stage_ms": k_ms / max(k_n, 1), "stages": k_n,
            "prof_steps": prof_steps, "tiles": tiles, "state": state, "t": t_reached}


def state_difference(ws, a, b):
    """Relative L1 and Linf of states a against b per kind of component
    (masses, momenta, energy, volume fractions) over every instance:
    L1 = sum |a - b| dV / sum |b| dV, Linf = max |a - b| / max |b|."""
    import numpy as np
    kinds = ("m", "rho_u", "rho_E", "alpha")
    num = dict.fromkeys(kinds, 0.0)
    den = dict.fromkeys(kinds, 0.0)
    mx = dict.fromkeys(kinds, 0.0)
    mref = dict.fromkeys(kinds, 0.0)
    for w, ua, ub in zip(ws, a, b):
        N, d = w.N, w.ndim
        ua = ua.reshape(w.nU, -1)
        ub = ub.reshape(w.nU, -1)
        vol = float(np.prod(w.dx))
        sl = {"m": slice(0, N), "rho_u": slice(N, N + d), "rho_E": slice(N + d, N + d + 1),
              "alpha": slice(N + d + 1, 2 * N + d + 1)}
        for k in kinds:
            diff = np.abs(ua[sl[k]] - ub[sl[k]])
            num[k] += diff.sum() * vol
            den[k] += np.abs(ub[sl[k]]).sum() * vol
            mx[k] = max(mx[k], float(diff.max()))
            mref[k] = max(mref[k], float(np.abs(ub[sl[k]]).max()))
    return {"L1_rel": {k: num[k] / den[k] for k in kinds},
            "Linf_rel": {k: mx[k] / mref[k] for k in kinds}}


def precision_pair(name, args, stream):
    """FP64 and mixed runs of one workload from the same initial state, and
    the difference of the mixed states from the FP64 states after the same
    K timed steps (each run with its own CFL steps).  Returns the summary and
    the two runs."""
    import numpy as np
    out = {}
    runs = {}
    for prec in ("fp64", "mixed"):
        ws = workload(name, prec)
        r = measure(ws, args, stream, keep_state=True)
        runs[prec] = (ws, r)
        out[prec] = {"value": r["value"], "unit": "cell-updates/s",
                     "ms_per_step": r["ms_per_step"], "stage_ms": r["stage_ms"]}
    ws, rf = runs["fp64"]
    _, rm = runs["mixed"]
    out["mixed_vs_fp64"] = dict(
        steps=args.steps, **state_difference(ws, rm["state"], rf["state"]),
        time_rel=float(np.abs(rm["t"] - rf["t"]).max() / np.abs(rf["t"]).max()))
    out["speedup_mixed"] = out["mixed"]["value"] / out["fp64"]["value"]
    for _, r in runs.values():
        r["state"] = None
    return out, runs


def pf_rate(name, precision, stream, steps):
    """The whole path per step: the hyperbolic step followed by the
    Phase-Field step (Eqs. (28), (4), (5)), same workload, eager steps (the
    solve checks convergence on the host), timed with events on the solver
    stream after two warm-up steps."""
    import torch
    from paper_2608_00746_amd.binding import MpWenoError, Solver
    ws = workload(name, precision)
    for w in ws:
        w.opts.phase_field = 1
    try:
        s = Solver(ws, stream=stream)
    except MpWenoError as err:
        return {"value": None, "note": str(err)}
    cells = sum(w.ncells for w in ws)
    s.advance(2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.advance(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    its = float(s.diag()[:, 29].max())
    s.close()
    return {"workload": name, "value": cells * steps / (ms / 1e3), "unit": "cell-updates/s",
            "ms_per_step": ms / steps, "steps": steps, "cg_iterations_last_step": its}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batched_256", choices=WORKLOADS)
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 / mixed comparison runs (profiling runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shapes (no mp_weno_autotune at set-up)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="copy a buffer of this many MiB device-to-device once before the "
                         "timed region (a reference kernel of known traffic for counters)")
    ap.add_argument("--tiles", default=None,
                    help="fixed tile shapes instead of the autotuner, as "
                         "x<lanes>/y<X>x<Y>/<plain|xcd> for every group, or a comma-separated "
                         "list of such, one per group of (d, N) in ascending order (the form "
                         "the bench line reports)")
    ap.add_argument("--pf-steps", type=int, default=10,
                    help="time this many steps of the 2048 x 1024 shock-bubble with the "
                         "Phase-Field step on (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.tiles is not None:
        # shapes by index into the library's candidate lists
        os.environ.update(tiles_env(args.tiles))
    from paper_2608_00746_amd import inputs as I
    ws = workload(args.workload, args.precision)
    precision = "mixed" if ws[0].opts.precision == I.PREC_MIXED else "fp64"
    stream = torch.cuda.Stream()
    cells = sum(w.ncells for w in ws)

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    comparison = {}
    if args.no_compare:
        r = measure(ws, args, stream)
    else:
        # the headline run is the pair's run of its precision
        summary, runs = precision_pair(args.workload, args, stream)
        comparison[args.workload] = summary
        ws, r = runs[precision]
    tk = tiles_key(args, ws, r["tiles"])
    bytes_stage = sum(8 * w.nU * w.ncells for w in ws) * (2 + 3 + 3) / 3.0
    stage_s = r["stage_ms"] / 1e3
    achieved = bytes_stage / stage_s / 1e9
    ctr = stage_counters(args.workload, precision, tk)
    roof = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": ctr["traffic"],
        "kernel": "RK stage: the sweep kernels of one stage over every instance",
        "bytes_per_launch": bytes_stage, "avg_launch_ms": r["stage_ms"],
        "launches": r["stages"],
        "timing": "HIP events around each RK stage on the solver stream, "
                  "%d eager steps after the timed region" % r["prof_steps"],
    }
    if ctr["flops64"] is not None:
        flops = (ctr["flops64"] + 0.5 * ctr["flops32"]) * cells
        tf = flops / stage_s / 1e12
        roof["alu"] = {
            "bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_PEAK_TFLOPS, "flops_per_launch": flops,
            "valu_issue_frac": ctr["valu"] * cells / stage_s / VALU_LANE_OPS_PEAK,
        }
    w0 = ws[0]
    out = {
        "metric": "cell-updates/s",
        "value": r["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": list(w0.n) if len(ws) == 1 else "uneven",
            "nphase": w0.N if len(ws) == 1 else sorted({w.N for w in ws}),
            "instances": len(ws), "cells": cells,
            "precision": precision,
            "recon": ["WENO-C", "WENO-CL", "WENO-JS", "WENO-W"][w0.opts.recon],
            "flux": ["HLLC", "HLL"][w0.opts.flux],
            "cfl": w0.opts.cfl, "graph": not args.no_graph,
            "tiles": tk,
        },
        "roofline": roof,
        "wall_s": r["wall_s"],
    }
    if len(ws) > 1:
        out["instances_per_s"] = len(ws) * args.steps / (r["ms_per_step"] * args.steps / 1e3)
    if not args.no_compare:
        if args.workload != "shock_bubble_2048x1024":
            comparison["shock_bubble_2048x1024"] = precision_pair(
                "shock_bubble_2048x1024", args, stream)[0]
        out["precision_comparison"] = comparison
    if args.pf_steps > 0:
        out["with_phase_field"] = pf_rate("shock_bubble_2048x1024", "fp64", stream,
                                          args.pf_steps)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(ws, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
