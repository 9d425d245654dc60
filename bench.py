"""Throughput of the WENO-C hyperbolic step on one MI355X.

A step is one full third-order SSP Runge-Kutta step (CFL time step on the
device, three RK stages) of every instance.  Default workload: the 2D
two-phase advection problem, 512 x 512 periodic, air bubble in water (SI),
FP64, WENO-C + HLLC, CFL 0.5.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME]
                  [--precision fp64|mixed] [--cpu-seconds S]

Inputs are synthetic and seeded (paper_2608_00746_amd.inputs) and resident in
HBM before the timed region.  The roofline entry reports the stage kernel
(x sweep + y sweep, + z sweep in 3D, of one RK stage) against both roofs, the one it is closer
to first:
* HBM: algorithmic bytes per launch (8 n_U bytes per cell read of the stage
  state, 8 n_U per cell read of the step-start state in stages 2 and 3, 8 n_U
  per cell written) over the average launch time;
* ALU: FP64 flops per launch (FP32 flops count half) over the average launch
  time against the FP64 vector peak, with the per-cell flop and VALU
  instruction counts of the counter table in profiles/ (per cell: every
  lane of a launch runs one cell's chain).
The launch time is measured with HIP events the library records on the
kernel's stream around each stage, in a short eager pass right after the
timed steps (those replay a captured graph, which cannot carry readable event
timestamps).  `traffic` is the measured HBM bytes per launch from the same
table, when it holds a row for this workload, tile choice and kernel source.

`with_phase_field` times the same workload with every step followed by the
Phase-Field step (the whole path of the method, Eqs. (28), (4) and (5)
included); `value` is the hyperbolic step alone, the workload as stated.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
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
    """Counter figures of one RK stage (x sweep + y sweep) from the table in
    profiles/ (rocprofv3 --pmc runs of this script):

    * traffic: HBM bytes per stage (FETCH_SIZE and WRITE_SIZE runs, scaled by
      a reference copy), only from the row of this workload, precision, tile
      choice and kernel source (else None);
    * flops64, flops32, valu: FP64 and FP32 flops and VALU lane-instructions
      per cell per stage (counted per launched lane: every lane runs one
      cell's chain), from the row of this tile choice, else the last row of
      this workload and precision."""
    out = {"traffic": None, "flops64": None, "flops32": None, "valu": None}
    if not os.path.exists(COUNTER_TABLE):
        return out
    key = kernel_source_hash()
    exact = False
    for line in open(COUNTER_TABLE):
        cols = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cols) != 9 or cols[0] in ("workload",) or cols[0].startswith("---"):
            continue
        wl, prec, tl, src, fetch_kib, write_kib, f64, f32, valu = cols
        if (wl, prec) != (workload, precision):
            continue
        if tl == tiles or not exact:
            out.update(flops64=float(f64), flops32=float(f32), valu=float(valu))
            exact = exact or tl == tiles
        if (tl, src) == (tiles, key):
            out["traffic"] = (float(fetch_kib) + float(write_kib)) * 1024.0
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


def cpu_baseline(ws, seconds):
    """The oracle as it stands, on the host cores, on a bounded sample: the
    first instance, whole steps until `seconds` have elapsed."""
    from oracle import mpo
    w = ws[0]
    o = w.opts
    pb = mpo.Problem(w.ndim, w.n, w.dx, w.bc, list(w.gamma), list(w.pinf), list(w.D),
                     list(w.pmin), list(w.cT), recon=o.recon, flux=o.flux, model=o.model,
                     energy_limiter=o.energy_limiter, cfl=o.cfl, t_end=0.0)
    U = w.U.reshape(-1).copy()
    t0 = time.perf_counter()
    steps = 0
    eta = o.eta_over_dx * min(w.dx)
    while True:
        if o.phase_field:
            U, _ = pb.step_pf(U, pb.dt(U, 0.0), eta)
        else:
            U = pb.step(U, pb.dt(U, 0.0))
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": steps * w.ncells / el, "unit": "cell-updates/s",
            "cores": mpo.num_threads(), "kind": "oracle",
            "sample": f"{steps} full RK3 steps{' with the Phase-Field step' if o.phase_field else ''} "
                      f"of {w.name} ({w.ncells} cells), "
                      f"{el:.1f} s, OpenMP over grid lines"}


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
    return {"value": cells * steps / (ms / 1e3), "unit": "cell-updates/s",
            "ms_per_step": ms / steps, "steps": steps,
            "cg_iterations_last_step": its}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="advection_2d_512",
                    choices=["advection_2d_512", "shock_bubble_2048x1024",
                             "shock_interface_n3_1024", "advection_1d_200", "batched_256",
                             "shock_vessel_bubble_400x200x200"])
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shapes (no mp_weno_autotune at set-up)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="copy a buffer of this many MiB device-to-device once before the "
                         "timed region (a reference kernel of known traffic for counters)")
    ap.add_argument("--tiles", default=None,
                    help="fixed tile shapes instead of the autotuner, as "
                         "x<lanes>/y<X>x<Y>/<plain|xcd> (the form the bench line reports)")
    ap.add_argument("--phase-field", action="store_true",
                    help="end every step with the Phase-Field step (reported separately)")
    ap.add_argument("--pf-steps", type=int, default=10,
                    help="after the main line's measurement, time this many steps of the "
                         "same workload with the Phase-Field step on (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2608_00746_amd.binding import Solver

    if args.tiles is not None:
        # shapes by index into the library's candidate lists
        xs, ys, sw = args.tiles.split("/")
        yx, yy = (int(v) for v in ys[1:].split("x"))
        os.environ["MPWENO_XSHAPE"] = str([256, 128, 64].index(int(xs[1:])))
        os.environ["MPWENO_YSHAPE"] = str([(16, 16), (32, 8), (16, 24), (0, 0)].index((yx, yy)) % 3)
        os.environ["MPWENO_XCD_SWIZZLE"] = {"plain": "0", "xcd": "1"}[sw]
    ws = workload(args.workload, args.precision)
    from paper_2608_00746_amd import inputs as I
    if args.phase_field:
        for w in ws:
            w.opts.phase_field = 1
    precision = "mixed" if ws[0].opts.precision == I.PREC_MIXED else "fp64"
    stream = torch.cuda.Stream()
    s = Solver(ws, stream=stream, use_graph=not args.no_graph)
    cells = sum(w.ncells for w in ws)
    tiles = None if (args.no_autotune or args.tiles) else s.autotune()

    s.advance(args.warmup)
    torch.cuda.synchronize()
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # timed region: K whole steps (mp_weno_advance: runs of 16 steps replay one
    # captured graph) bracketed by synchronisation and by events on the
    # solver's stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.advance(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)

    # the stage kernels (x sweep + y (+ z) sweep of one RK stage) timed by HIP event
    # pairs the library records on its stream around each stage; a graph
    # cannot carry readable event timestamps, so these steps are launched
    # eagerly right after the timed region, from the state it left
    prof_steps = max(1, min(args.steps, 20))
    s.profile(3)
    for _ in range(prof_steps):
        s.step()
    k_ms, k_n = s.timing(reset=True)
    s.profile(0)

    # sanity: the state stayed finite and admissible
    d = s.diag()
    cg_its = float(d[:, 29].max())
    if (d[:, 25] > 0).any():
        raise SystemExit("non-finite state after the timed steps")

    ms_step = ms / args.steps
    value = cells * args.steps / (ms / 1e3)
    bytes_launch = sum(8 * w.nU * w.ncells for w in ws) * (2 + 3 + 3) / 3.0
    avg_launch_s = (k_ms / 1e3) / max(k_n, 1)
    achieved = bytes_launch / avg_launch_s / 1e9
    tiles_key = args.tiles if args.tiles else "default" if tiles is None else ",".join(
        sorted({"x%d/y%dx%d/%s" % (t[0], t[1], t[2], "xcd" if t[3] else "plain")
                for t in tiles.tolist()}))
    ctr = stage_counters(args.workload, precision, tiles_key)
    hbm = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": ctr["traffic"],
        "bytes_per_launch": bytes_launch,
    }
    roof = hbm
    if ctr["flops64"] is not None:
        # FP64-equivalent flops: an FP32 flop takes half an FP64 slot
        flops = (ctr["flops64"] + 0.5 * ctr["flops32"]) * cells
        tf = flops / avg_launch_s / 1e12
        alu = {
            "bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS, "traffic": ctr["traffic"],
            "flops_per_launch": flops,
            "valu_issue_frac": ctr["valu"] * cells / avg_launch_s / VALU_LANE_OPS_PEAK,
        }
        # the roof the stage is closer to binds it
        if alu["frac"] > hbm["frac"]:
            roof = dict(alu, hbm=hbm)
        else:
            roof = dict(hbm, alu=alu)
    roof.update({
        "kernel": "RK stage (x sweep + transverse sweeps)",
        "avg_launch_ms": avg_launch_s * 1e3, "launches": k_n,
        "timing": "HIP events around each RK stage on the solver stream, "
                  "%d eager steps after the timed region" % prof_steps,
    })
    w0 = ws[0]
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
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
            "recon": ["WENO-C", "WENO-CL"][w0.opts.recon],
            "flux": ["HLLC", "HLL"][w0.opts.flux],
            "cfl": w0.opts.cfl, "graph": not args.no_graph and not args.phase_field,
            "phase_field": bool(args.phase_field),
            "tiles": [args.tiles] if args.tiles else "default" if tiles is None else
                     sorted({"x%d/y%dx%d/%s" % (t[0], t[1], t[2], "xcd" if t[3] else "plain")
                             for t in tiles.tolist()}),
        },
        "roofline": roof,
        "wall_s": wall,
    }
    if len(ws) > 1:
        out["instances_per_s"] = len(ws) * args.steps / (ms / 1e3)
    if args.phase_field:
        out["pf_cg_iterations_last_step"] = cg_its
    s.close()
    if args.pf_steps > 0 and not args.phase_field:
        out["with_phase_field"] = pf_rate(args.workload, args.precision, stream, args.pf_steps)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(ws, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
