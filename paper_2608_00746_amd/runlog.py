"""Run a context in blocks of steps and log one JSON line per block.

Each line holds, per instance, the paper's diagnostics that the GPU reduces
(Sec. 4: the sum-alpha error, the bounds of Eq. (8), psi of Eq. (9), the
conservation of mass, momentum and energy against the first line, and the
interface thickness N_I of Eq. (30) for alpha_1), the time and step count,
and for the block its throughput: cell-updates/s, ms per step and the
fraction of the HBM roofline on algorithmic bytes (8 n_U doubles per
cell-update: one RK3 step reads and writes the state three times and reads
U^n twice).  Rows also carry the precision, phases, dimensions, workload
names and the git revision, so that lines of different runs can be told
apart.  Callers may add fields of their own per line (`extra`, e.g. errors
against an exact solution that only they know).
"""
from __future__ import annotations

import json
import os
import subprocess
import time

import numpy as np

HBM_PEAK_BYTES = 8.0e12      # MI355X HBM3E, bytes/s

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def git_revision():
    """HEAD of the repository this package sits in, or None."""
    try:
        r = subprocess.run(["git", "-C", ROOT, "rev-parse", "--short=12", "HEAD"],
                           capture_output=True, text=True, timeout=10)
    except (OSError, subprocess.SubprocessError):
        return None
    rev = r.stdout.strip()
    return rev if r.returncode == 0 and rev else None


def instance_record(w, d, tot0):
    """Diagnostics of one instance: w its Workload, d its diagnostics row,
    tot0 its totals (slots 0 .. n_U - 1) of the first line."""
    N, D = w.N, w.ndim
    tot = d[:w.nU]
    cons = []
    for c in range(N + D + 1):          # m_p, rho u_k, rho E
        ref = abs(tot0[c]) if tot0[c] != 0.0 else 1.0
        cons.append(float(abs(tot[c] - tot0[c]) / ref))
    den = min(w.dx) * d[33]
    return {
        "name": w.name, "t": float(d[26]), "steps": int(d[27]),
        "sum_alpha_err": float(d[20]), "min_m": float(d[21]),
        "min_alpha": float(d[22]), "max_alpha": float(d[23]),
        "min_psi": float(d[24]), "nonfinite": int(d[25]),
        "conservation_rel": cons,
        "interface_thickness": float(d[32] / den) if den > 0.0 else 0.0,
        "cg_iterations": float(d[29]), "cg_residual": float(d[30]),
    }


def run(solver, nsteps, every, path, extra=None, sync=None):
    """Advance `solver` (binding.Solver or any object with its advance,
    diag, w and opts) by nsteps in blocks of `every`, appending one JSON
    line per block (and one before the first) to `path`.  extra(solver,
    step) -> dict adds caller fields.  sync() waits for the GPU before the
    clock is read (default: torch.cuda.synchronize when torch is loaded).
    Returns the records written."""
    if every <= 0 or nsteps < 0:
        raise ValueError("every must be positive and nsteps non-negative")
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    ws = list(solver.w)
    cells = float(sum(w.ncells for w in ws))
    bytes_per_step = float(sum(8 * 8 * w.nU * w.ncells for w in ws))
    head = {
        "precision": "mixed" if solver.opts.precision == 1 else "fp64",
        "N": sorted({w.N for w in ws}), "d": sorted({w.ndim for w in ws}),
        "instances": len(ws), "cells": int(cells), "workloads": sorted({w.name for w in ws}),
        "recon": int(solver.opts.recon), "flux": int(solver.opts.flux),
        "cfl": float(solver.opts.cfl), "phase_field": bool(solver.opts.phase_field),
        "git": git_revision(),
    }
    d0 = np.asarray(solver.diag())
    tot0 = [d0[i, :w.nU].copy() for i, w in enumerate(ws)]
    out = []
    done = 0
    block_s = None
    n_block = 0

    def emit():
        d = np.asarray(solver.diag())
        rec = dict(head)
        rec["step"] = done
        if block_s is not None and n_block > 0:
            rec["ms_per_step"] = 1e3 * block_s / n_block
            rec["cell_updates_per_s"] = cells * n_block / block_s
            rec["hbm_frac_algorithmic"] = bytes_per_step * n_block / block_s / HBM_PEAK_BYTES
        rec["instances_diag"] = [instance_record(w, d[i], tot0[i]) for i, w in enumerate(ws)]
        if extra is not None:
            rec.update(extra(solver, done))
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")
        out.append(rec)

    emit()
    while done < nsteps:
        n_block = min(every, nsteps - done)
        sync()
        t0 = time.perf_counter()
        solver.advance(n_block)
        sync()
        block_s = time.perf_counter() - t0
        done += n_block
        emit()
    return out
