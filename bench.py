#!/usr/bin/env python3
"""Throughput benchmark of the finite-element Bloch-Torrey hot path on one MI355X.

A step is one whole simulation of the workload: every (b, direction) system
is stepped from t = 0 to the echo time with the theta-scheme (right-hand
side, initial guess, Krylov solve per step) and its signal is integrated.
The default workload is the batched two-compartment case: a z-cylinder of
radius 5 um in a 12 um periodic box on a 57^3-cube Kuhn mesh (195,112 nodes,
196,593 DOFs), 64 Fibonacci directions x 16 b-values in [0, 5000] s/mm^2 =
1024 systems solved in one batch, PGSE delta = 10.6 ms, Delta = 13.4 ms,
dt = 100 us (240 steps).

Prints one JSON line:
  value      DOF-steps/s = n_dof x n_systems x n_steps / seconds per step
  roofline   the dominant kernel's algorithmic HBM bytes per launch over its
             mean launch time (HIP events on the library's stream), vs 8 TB/s
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = {"spmv": 1, "update": 2, "pupdate": 3, "init": 4}


def workload(name):
    import dmri_inputs as di
    if name == "config2":
        prob, seq, sysl = di.config2()
        desc = ("cylinder r=5um in 12um periodic box, 57^3 Kuhn cubes, 2 compartments, "
                "kappa=1e-5, 64 dirs x 16 b in [0,5000]")
    elif name == "config1":
        prob, seq, sysl = di.config1()
        desc = "cylinder r=5um in 12um periodic box, 36^3 Kuhn cubes, 8 b in [0,3000] along x"
    elif name == "config0":
        prob, seq, sysl = di.config0()
        desc = "free diffusion [-5,5]^3, 10^3 Kuhn cubes, b=1000 along x"
    else:
        raise SystemExit("unknown workload %s" % name)
    return prob, seq, sysl, desc


def kernel_bytes(kind, n_dof, nnz, total_iters, tile, prec_bytes, n_steps, n_sys):
    """Algorithmic HBM bytes of one kernel summed over a run.

    Vector traffic per DOF and system (complex of 2*prec_bytes) and matrix
    traffic per matrix row per active system tile (every tile of S systems
    re-reads the matrix): see the design doc for the derivation.
    """
    c = 2 * prec_bytes
    mat = nnz * (4 + 5 * prec_bytes) + 4 * n_dof       # col + K0 + {MD, Vx, Vy, Vz} + row_ptr
    diag = n_dof * 5 * prec_bytes
    tile_iters = total_iters / tile
    if kind == "spmv":
        return 2 * c * n_dof * total_iters + mat * tile_iters
    if kind == "update":
        return 6 * c * n_dof * total_iters + diag * tile_iters
    if kind == "pupdate":
        return 3 * c * n_dof * total_iters + diag * tile_iters
    if kind == "init":
        # gathers u_prev (and u_prev2), writes x, r, p, reads both base arrays
        return (5 * c * n_dof * n_sys + (mat + nnz * prec_bytes) * n_sys / tile) * n_steps
    raise ValueError(kind)


def cpu_baseline(prob, seq, sysl, n_steps_sample):
    """FP64 oracle (assembly + Krylov-to-rounding solves) on a bounded sample."""
    from oracle import fem, timestep
    t0 = time.perf_counter()
    asm = fem.assemble(prob)
    t_asm = time.perf_counter() - t0
    i = int(np.argmax(sysl.b))
    t0 = time.perf_counter()
    timestep.solve_transformed(asm, seq, float(sysl.b[i]), sysl.q[i], n_steps=n_steps_sample,
                               solver="krylov")
    t_run = time.perf_counter() - t0
    rate = asm.n_dof * n_steps_sample / t_run
    return {
        "value": rate, "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
        "sample": ("1 system (b=%g) x first %d of %d steps, single-threaded SciPy CG to 1e-13; "
                   "assembly %.1fs excluded" % (sysl.b[i], n_steps_sample, seq.n_steps, t_asm)),
        "host_cpus": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2", choices=["config0", "config1", "config2"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--guess", type=int, default=1)
    ap.add_argument("--time-kernel", default="spmv", choices=sorted(KERNELS))
    ap.add_argument("--sys-tile", type=int, default=0)
    ap.add_argument("--blocks-per-xcd", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--progress", type=int, default=40, help="library progress line every k steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (got --gpus %d); the per-GPU "
              "shard design is described in DESIGN.md" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_01719_amd import Simulator

    prob, seq, sysl, desc = workload(args.workload)
    prec = {"fp64": 0, "mixed": 1, "fp32": 2}[args.precision]
    rtol = args.rtol if args.rtol is not None else {0: 1e-10, 1: 1e-10, 2: 1e-6}[prec]
    print("bench: workload %s (%s), %d systems, precision %s" % (
        args.workload, desc, len(sysl), args.precision), file=sys.stderr, flush=True)

    sim = Simulator(0)
    sim.set_sequence(seq)
    t0 = time.perf_counter()
    pid = sim.add_problem(prob)
    t_asm = time.perf_counter() - t0
    n_dof, nnz = sim.dmri_problem_info(pid)
    opts = dict(precision=prec, rtol=rtol, guess=args.guess,
                time_kernel=KERNELS[args.time_kernel], progress=args.progress)
    if args.sys_tile:
        opts["sys_tile"] = args.sys_tile
    if args.blocks_per_xcd:
        opts["blocks_per_xcd"] = args.blocks_per_xcd
    sim.set_options(**opts)
    pids = np.full(len(sysl), pid, np.int32)

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        bcopy = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            bcopy.copy_(a)
        torch.cuda.synchronize()
        del a, bcopy

    for w in range(args.warmup):
        sig, st = sim.dmri_run(pids, sysl.b, sysl.q)
        print("bench: warmup %d done (%.2fs solve)" % (w, st["t_solve_s"]), file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    tot_iters = 0
    t_kernel = 0.0
    n_launch = 0
    for k in range(args.steps):
        sig, st = sim.dmri_run(pids, sysl.b, sysl.q)
        tot_iters += st["total_iterations"]
        t_kernel += st["t_kernel_s"]
        n_launch += st["n_kernel_launches"]
        print("bench: step %d done (%.2fs solve, %d iterations)" % (
            k, st["t_solve_s"], st["total_iterations"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    ms_per_step = 1e3 * elapsed / args.steps
    n_steps = st["n_steps"]
    value = n_dof * len(sysl) * n_steps * args.steps / elapsed

    tile = args.sys_tile or (64 if len(sysl) >= 64 else 32 if len(sysl) >= 32 else
                             16 if len(sysl) >= 16 else 8)
    pbytes = 8 if prec == 0 else 4
    kb = kernel_bytes(args.time_kernel, n_dof, nnz, tot_iters, tile, pbytes, n_steps * args.steps,
                      len(sysl))
    achieved = kb / t_kernel / 1e9 if t_kernel > 0 else None
    roofline = {
        "kernel": {"spmv": "k_spmv_dot", "update": "k_update", "pupdate": "k_pupdate",
                   "init": "k_init"}[args.time_kernel],
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
        "launches": n_launch, "mean_launch_us": 1e6 * t_kernel / max(1, n_launch),
        "bytes_per_launch": kb / max(1, n_launch),
    }
    out = {
        "metric": "DOF-steps/s", "value": value, "unit": "DOF-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "f32+f64", 2: "f32"}[prec], "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n_dof": n_dof, "nnz": nnz,
                   "n_systems": len(sysl), "time_steps": n_steps, "dt_us": seq.dt,
                   "rtol": rtol, "guess": args.guess, "sys_tile": tile,
                   "parallelism": "single GPU, systems batched"},
        "time_to_signal_s_per_pair": elapsed / args.steps / len(sysl),
        "krylov_iterations_per_system_step": tot_iters / (len(sysl) * n_steps * args.steps),
        "host_assembly_s": t_asm,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, seq, sysl, args.cpu_steps)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
