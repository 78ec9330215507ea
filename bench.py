#!/usr/bin/env python3
"""Throughput benchmark of the finite-element Bloch-Torrey hot path on one MI355X.

A step is one whole simulation of the workload: every (b, direction) system
is stepped from t = 0 to the echo time with the theta-scheme (right-hand
side, initial guess, Krylov solve per step) and its signal is integrated.
The default workload is the batched two-compartment case: a z-cylinder of
radius 5 um in a 12 um periodic box on a 57^3-cube Kuhn mesh (195,112 nodes,
196,593 DOFs), 64 Fibonacci directions x 16 b-values in [0, 5000] s/mm^2 =
1024 systems solved in one batch, PGSE delta = 10.6 ms, Delta = 13.4 ms,
dt = 100 us (240 steps). The default solver is the mixed-precision form
(FP32 matrices and Krylov vectors, FP64 dots, FP64 residual refinement and
signal) at a per-step relative residual of 1e-6, which keeps every signal
within 1e-5 of the all-FP64 solution (the accuracy target is 1e-4).

Prints one JSON line:
  value      DOF-steps/s = n_dof x n_systems x n_steps / seconds per step
  roofline   the dominant kernel's algorithmic HBM bytes per launch over its
             mean launch time (HIP events on the library's stream), vs 8 TB/s
  plain_fp64 the plain FP64 GPU solve (one system at a time, previous-step
             guess, all FP64, same tolerance) on a sample of the systems
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

# The CPU oracle baseline runs one single-threaded process per core; BLAS
# thread pools must be sized before numpy is imported.
for _k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_k] = "1"

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS = {"spmv": 1, "update": 2, "pupdate": 3, "init": 4}
KERNEL_NAMES = {"spmv": "k_spmv_dot", "update": "k_update", "pupdate": "k_pupdate",
                "init": "k_init"}


def workload(name):
    """(sequence, [(problem, systems), ...], description, golden fixtures)."""
    import dmri_inputs as di
    if name == "cylinder_57_batched":
        prob, seq, sysl = di.cylinder_57_batched()
        desc = ("cylinder r=5um in 12um periodic box, 57^3 Kuhn cubes, 2 compartments, "
                "kappa=1e-5, 64 dirs x 16 b in [0,5000]")
        return seq, [(prob, sysl)], desc, {0: "cylinder_57_full"}
    if name == "cylinder_36":
        prob, seq, sysl = di.cylinder_36()
        desc = "cylinder r=5um in 12um periodic box, 36^3 Kuhn cubes, 8 b in [0,3000] along x"
        return seq, [(prob, sysl)], desc, {0: "cylinder_36"}
    if name == "free_diffusion_10":
        prob, seq, sysl = di.free_diffusion_10()
        desc = "free diffusion [-5,5]^3, 10^3 Kuhn cubes, b=1000 along x"
        return seq, [(prob, sysl)], desc, {}
    if name == "seeded_cells_batch":
        items = []
        for seed in range(8):
            prob, seq, sysl = di.seeded_cells(seed)
            items.append((prob, sysl))
        desc = ("8 seeded geometries (seeds 0-7) of 5-30 cylinders/spheres in a 30um periodic "
                "box, 39^3-93^3 Kuhn cubes, kappa log-uniform 1e-6..1e-4, 32 (b, dir) pairs each")
        return seq, items, desc, {2: "seeded_cells_seed2", 3: "seeded_cells_seed3"}
    raise SystemExit("unknown workload %s" % name)


def golden_error(fixtures, sigs):
    """Largest relative error of the run's signals against the oracle's stored
    signals (tests/golden/, written from the CPU oracle only), floor 1e-8 of the
    b = 0 signal (the total initial magnetization)."""
    import json
    worst, n = 0.0, 0
    for item, name in fixtures.items():
        with open(os.path.join(ROOT, "tests", "golden", name + ".json")) as f:
            d = json.load(f)
        ref = np.array(d["signal_re"]) + 1j * np.array(d["signal_im"])
        got = sigs[item][np.array(d["index"])]
        floor = 1e-8 * np.abs(ref).max()
        worst = max(worst, float((np.abs(got - ref) / np.maximum(np.abs(ref), floor)).max()))
        n += len(ref)
    return {"max_rel_err": worst, "n_signals": n, "fixtures": sorted(fixtures.values())} if n \
        else None


def kernel_bytes(kind, n_dof, nnz, total_iters, tile, prec_bytes, n_steps, n_sys, cp=None):
    """Algorithmic HBM bytes of one kernel summed over a run.

    Vector traffic per DOF and system (complex of c = 2*prec_bytes bytes; the
    search direction p may be stored narrower, cp bytes per complex: BF16
    directions of the paired inner solves, 4 B) plus matrix traffic per active
    system tile, since every tile of S systems re-reads the matrix: the SpMV
    reads p once and writes q (cp + c) and reads per stored entry a column
    index (4 B) and five values (K0, M_D, V_x, V_y, V_z), plus the row
    pointers; the CG update reads r, q and writes r (3c); the direction update
    reads r, p, x and writes p, x (3c + 2cp); both read the five diagonal
    values per row and tile.
    """
    c = 2 * prec_bytes
    cp = c if cp is None else cp
    mat = nnz * (4 + 5 * prec_bytes) + 4 * n_dof       # col + K0 + {MD, Vx, Vy, Vz} + row_ptr
    diag = n_dof * 5 * prec_bytes
    tile_iters = total_iters / tile
    if kind == "spmv":
        return (cp + c) * n_dof * total_iters + mat * tile_iters
    if kind == "update":  # r, q read, r written
        return 3 * c * n_dof * total_iters + diag * tile_iters
    if kind == "pupdate":  # r, p, x read, p, x written
        return (3 * c + 2 * cp) * n_dof * total_iters + diag * tile_iters
    if kind == "init":
        # gathers u_prev (and u_prev2), writes x, r, p, reads both base arrays
        return (5 * c * n_dof * n_sys + (mat + nnz * prec_bytes) * n_sys / tile) * n_steps
    raise ValueError(kind)


def profiled_traffic(kernel, workload, precision, rtol, key="traffic_bytes_per_launch"):
    """Measured HBM bytes per launch of `kernel` from the committed rocprofv3
    counter summary (`key`: the copy-calibrated FETCH + WRITE figure, or
    traffic_l2_miss_bytes_per_launch), or None when none matches or the
    library sources changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", "hbm_counters_%s_%s_%s.md" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_t = re.search(key + r":\s*([0-9.eE+]+)", text)
    m_h = re.search(r"csrc_sha256:\s*([0-9a-f]+)", text)
    m_w = re.search(r"workload: \S+ precision=\S+ rtol=(\S+)", text)
    if not (m_t and m_h and m_w) or float(m_w.group(1)) != rtol:
        return None
    if csrc_sha256() != m_h.group(1):
        return None
    return float(m_t.group(1))


def csrc_sha256():
    """SHA-256 over the library sources (kernels and the host code that shapes
    the launches and the DOF order), in name order."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1908_01719_amd", "csrc", "*"))):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(os.path.basename(f).encode())
            h.update(open(f, "rb").read())
    return h.hexdigest()


_CPU = {}


def _cpu_worker(args):
    """One single-threaded oracle solve of n steps of one system, from step s0."""
    i, s0, n_steps = args
    from oracle import timestep
    asm, seq, sysl = _CPU["asm"], _CPU["seq"], _CPU["sysl"]
    t0 = time.perf_counter()
    timestep.solve_transformed(asm, seq, float(sysl.b[i]), sysl.q[i], n_steps=n_steps,
                               solver="krylov", start_step=s0)
    return time.perf_counter() - t0


def cpu_sample_plan(sysl, n_total_steps, n_steps_sample, n_proc):
    """(system, first step) per oracle process: systems spread over the b range
    (sorted by b, evenly spaced), windows of n_steps_sample steps spread over
    the whole echo, so the sample mixes easy and hard solves as the full run
    does."""
    order = np.argsort(np.asarray(sysl.b), kind="stable")
    plan = []
    for k in range(n_proc):
        i = int(order[(2 * k + 1) * len(order) // (2 * n_proc)])
        s0 = (k * (n_total_steps - n_steps_sample)) // max(1, n_proc - 1)
        plan.append((i, int(s0)))
    return plan


def cpu_baseline(prob, seq, sysl, n_steps_sample, n_proc):
    """FP64 oracle (assembly + Krylov-to-rounding solves) on a bounded sample:
    n_proc single-threaded processes, each stepping a different system over a
    different window of the echo."""
    import multiprocessing as mp
    from oracle import fem
    t0 = time.perf_counter()
    asm = fem.assemble(prob)
    t_asm = time.perf_counter() - t0
    _CPU.update(asm=asm, seq=seq, sysl=sysl)
    plan = cpu_sample_plan(sysl, seq.n_steps, n_steps_sample, n_proc)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(n_proc) as pool:
        per = pool.map(_cpu_worker, [(i, s0, n_steps_sample) for i, s0 in plan])
    wall = time.perf_counter() - t0
    rate = asm.n_dof * n_steps_sample * n_proc / wall
    return {
        "value": rate, "unit": "DOF-steps/s", "cores": n_proc, "kind": "oracle",
        "sample": ("%d systems spread over b (%g..%g) x %d-step windows spread over the %d-step "
                   "echo (first steps %s), each started from the initial magnetization; one "
                   "single-threaded process each (SciPy CG to 1e-13, Jacobi); wall %.1fs; "
                   "per-process %.1f-%.1fs; assembly %.1fs excluded"
                   % (n_proc, min(float(sysl.b[i]) for i, _ in plan),
                      max(float(sysl.b[i]) for i, _ in plan), n_steps_sample, seq.n_steps,
                      [s for _, s in plan], wall, min(per), max(per), t_asm)),
        "host_cpus": os.cpu_count(),
    }


def plain_fp64(sim, pid, sysl, rtol, n_sample, batched_sig):
    """Plain FP64 GPU solve, one system at a time, previous-step guess."""
    order = np.argsort(-np.asarray(sysl.b), kind="stable")
    pick = [int(order[k * len(order) // n_sample]) for k in range(n_sample)]
    saved = {k: sim.dmri_get_option(k) for k in ("precision", "rtol", "guess", "time_kernel",
                                                  "progress")}
    sim.set_options(precision=0, rtol=rtol, guess=0, time_kernel=0, progress=0)
    t = []
    diff = []
    for i in pick:
        t0 = time.perf_counter()
        sig, _ = sim.dmri_run([pid], sysl.b[i:i + 1], sysl.q[i:i + 1])
        t.append(time.perf_counter() - t0)
        diff.append(abs(sig[0] - batched_sig[i]) / abs(sig[0]))
    sim.set_options(**saved)
    return {
        "time_to_signal_s_per_pair": float(np.mean(t)),
        "sample": "%d systems, indices %s (b = %s), rtol %g" % (
            n_sample, pick, [float(sysl.b[i]) for i in pick], rtol),
        "max_rel_diff_vs_batched": float(max(diff)),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cylinder_57_batched",
                    choices=["free_diffusion_10", "cylinder_36", "cylinder_57_batched",
                             "seeded_cells_batch"])
    ap.add_argument("--precision", default="mixed", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--guess", type=int, default=1)
    ap.add_argument("--time-kernel", default="spmv", choices=sorted(KERNELS))
    ap.add_argument("--sys-tile", type=int, default=0)
    ap.add_argument("--blocks-per-xcd", type=int, default=0)
    ap.add_argument("--mesh-merge", type=int, default=None,
                    help="several meshes as one batch, every launch over all of them "
                         "(library option mesh_merge; default: on for seeded_cells_batch)")
    ap.add_argument("--autotune", type=int, default=None,
                    help="library autotuner (default: on for a several-mesh workload run mesh "
                         "by mesh)")
    ap.add_argument("--concurrency", type=int, default=1,
                    help="problems of a multi-mesh workload run at once (lanes)")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes for the CPU baseline (0 = min(16, host CPUs))")
    ap.add_argument("--plain-sample", type=int, default=4,
                    help="systems timed one at a time in plain FP64 (0 = skip)")
    ap.add_argument("--progress", type=int, default=40, help="library progress line every k steps")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                    help="extra library option (set before the meshes are added, so DOF "
                         "ordering options apply)")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="stop every run after this many time steps (profiling aid; the "
                         "value line is then not the full-echo workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy and a 1 GiB gather of 1 KiB rows "
                         "in random order (for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (got --gpus %d); systems and "
              "meshes would shard across GPUs without communication, but only one GPU is "
              "driven here" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_01719_amd import Simulator

    seq, items, desc, fixtures = workload(args.workload)
    n_pairs = sum(len(sl) for _, sl in items)
    prec = {"fp64": 0, "mixed": 1, "fp32": 2}[args.precision]
    rtol = args.rtol if args.rtol is not None else 1e-6
    merge = args.mesh_merge if args.mesh_merge is not None else int(len(items) > 1)
    autotune = args.autotune if args.autotune is not None else int(len(items) > 1 and not merge)
    print("bench: workload %s (%s), %d systems on %d meshes, precision %s" % (
        args.workload, desc, n_pairs, len(items), args.precision), file=sys.stderr, flush=True)

    # The oracle's worker processes are forked before this process touches the GPU.
    # A multi-mesh workload is sampled on its smallest mesh.
    cpu = None
    if not args.no_cpu_baseline:
        n_proc = args.cpu_procs or min(16, os.cpu_count() or 1)
        small = min(range(len(items)), key=lambda i: items[i][0].n_nodes)
        print("bench: timing the CPU oracle on a bounded sample (%d processes)" % n_proc,
              file=sys.stderr, flush=True)
        cpu = cpu_baseline(items[small][0], seq, items[small][1], args.cpu_steps, n_proc)
        if len(items) > 1:
            cpu["sample"] = "mesh %d of %d (the smallest): %s" % (small, len(items), cpu["sample"])
        print("bench: CPU oracle %.3g DOF-steps/s" % cpu["value"], file=sys.stderr, flush=True)

    sim = Simulator(0)
    sim.set_sequence(seq)
    extra = {kv.split("=")[0]: float(kv.split("=")[1]) for kv in args.opt}
    sim.set_options(**extra)
    t0 = time.perf_counter()
    pid_list = [sim.add_problem(prob) for prob, _ in items]
    t_asm = time.perf_counter() - t0
    info = [sim.dmri_problem_info(p) for p in pid_list]
    opts = dict(precision=prec, rtol=rtol, guess=args.guess, autotune=autotune,
                concurrency=args.concurrency, mesh_merge=merge,
                time_kernel=KERNELS[args.time_kernel], progress=args.progress)
    if args.sys_tile:
        opts["sys_tile"] = args.sys_tile
    if args.blocks_per_xcd:
        opts["blocks_per_xcd"] = args.blocks_per_xcd
    if args.time_steps:
        opts["n_steps"] = args.time_steps
        opts["signal"] = 0
    opts.update(extra)
    sim.set_options(**opts)
    pids = np.concatenate([np.full(len(sl), p, np.int32) for p, (_, sl) in zip(pid_list, items)])
    bs = np.concatenate([sl.b for _, sl in items])
    qs = np.concatenate([sl.q for _, sl in items])
    owner = np.concatenate([np.full(len(sl), i) for i, (_, sl) in enumerate(items)])

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        bcopy = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            torch.mul(a, 2.0, out=bcopy)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        del a, bcopy
        # Gather leg: 1 KiB rows in a seeded random order (the SpMV's access
        # shape: whole rows of a tile, in an order set by the mesh), each
        # source row read once: 1 GiB gathered, 1 GiB written.
        src = torch.empty((1 << 20, 256), dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        gen = torch.Generator(device="cpu")
        gen.manual_seed(0)
        perm = torch.randperm(1 << 20, generator=gen).to("cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.index_select(src, 0, perm, out=dst)
        torch.cuda.synchronize()
        del src, dst, perm

    for w in range(args.warmup):
        sig, st = sim.dmri_run(pids, bs, qs)
        print("bench: warmup %d done (%.2fs solve)" % (w, st["t_solve_s"]), file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    iters_item = np.zeros(len(items))
    t_kernel = 0.0
    n_launch = 0
    tot_iters = 0
    for k in range(args.steps):
        sig, st = sim.dmri_run(pids, bs, qs)
        tot_iters += st["total_iterations"]
        t_kernel += st["t_kernel_s"]
        n_launch += st["n_kernel_launches"]
        iters_item += np.bincount(owner, weights=st["iters_total"], minlength=len(items))
        print("bench: step %d done (%.2fs solve, %d iterations)" % (
            k, st["t_solve_s"], st["total_iterations"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    ms_per_step = 1e3 * elapsed / args.steps
    n_steps = st["n_steps"]
    dof_sys = sum(info[i][0] * len(sl) for i, (_, sl) in enumerate(items))
    value = dof_sys * n_steps * args.steps / elapsed

    # Algorithmic bytes of the timed kernel, summed over the meshes.
    pbytes = 8 if prec == 0 else 4
    kb = 0.0
    tiles = []
    paired_any = False
    for i, (_, sl) in enumerate(items):
        ns = len(sl)
        tile = args.sys_tile or (64 if ns >= 64 else 32 if ns >= 32 else 16 if ns >= 16 else 8)
        if autotune and not args.sys_tile and sim.dmri_get_option("tuned_sys_tile") > 0:
            tile = min(tile, int(sim.dmri_get_option("tuned_sys_tile")))
        # Mixed precision on more than 64 systems runs its FP32 Krylov kernels on
        # 128-system paired-lane tiles (the matrix is read once per such tile).
        paired = (prec == 1 and tile == 64 and ns > 64
                  and sim.dmri_get_option("pair_lanes") == 1 and args.time_kernel != "init")
        paired_any |= paired
        ktile = 128 if paired else tile
        tiles.append(ktile)
        # paired inner solves keep their search directions in BF16 (option dir_bf16)
        cp = 4 if (paired and sim.dmri_get_option("dir_bf16") == 1) else None
        kb += kernel_bytes(args.time_kernel, info[i][0], info[i][1], iters_item[i], ktile, pbytes,
                           n_steps * args.steps, ns, cp)
    kname = KERNEL_NAMES[args.time_kernel]
    if paired_any:
        kname = kname.replace("k_spmv_dot", "k_spmv_pair").replace("k_update", "k_update_pair") \
            .replace("k_pupdate", "k_pupdate_pair")
    achieved = kb / t_kernel / 1e9 if t_kernel > 0 else None
    roofline = {
        "kernel": kname,
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
        "traffic": profiled_traffic(kname, args.workload, args.precision, rtol),
        "traffic_l2_miss": profiled_traffic(kname, args.workload, args.precision, rtol,
                                            "traffic_l2_miss_bytes_per_launch"),
        "launches": n_launch, "mean_launch_us": 1e6 * t_kernel / max(1, n_launch),
        "bytes_per_launch": kb / max(1, n_launch),
        "traffic_unit": "bytes per launch: traffic = rocprofv3 FETCH_SIZE x2 + WRITE_SIZE "
                        "(copy-calibrated); traffic_l2_miss = TCC_MISS x 64 B + WRITE_SIZE",
    }
    sigs = [sig[owner == i] for i in range(len(items))]
    config = {"workload": args.workload, "description": desc,
              "n_dof": [int(x[0]) for x in info] if len(items) > 1 else int(info[0][0]),
              "nnz": [int(x[1]) for x in info] if len(items) > 1 else int(info[0][1]),
              "n_systems": n_pairs, "time_steps": n_steps, "dt_us": seq.dt,
              "rtol": rtol, "guess": args.guess,
              "extrap_order": int(sim.dmri_get_option("extrap_order")),
              "sys_tile": tiles if len(items) > 1 else tiles[0], "autotune": autotune,
              "concurrency": args.concurrency, "mesh_merge": merge, "extra_options": extra,
              "parallelism": ("single GPU, all meshes in one batch" if merge and len(items) > 1
                              else "single GPU, systems batched per mesh")}
    out = {
        "metric": "DOF-steps/s", "value": value, "unit": "DOF-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "f32+f64", 2: "f32"}[prec], "data": "synthetic",
        "config": config,
        "time_to_signal_s_per_pair": elapsed / args.steps / n_pairs,
        "krylov_iterations_per_system_step": tot_iters / (n_pairs * n_steps * args.steps),
        "accuracy_vs_oracle": golden_error(fixtures, sigs) if n_steps == seq.n_steps else None,
        "host_assembly_s": t_asm,
        "roofline": roofline,
        "plain_fp64": None,
        "cpu_baseline": None,
    }
    if args.plain_sample > 0 and len(items) == 1:
        print("bench: timing the plain FP64 solve on %d systems" % args.plain_sample,
              file=sys.stderr, flush=True)
        sim.set_options(autotune=0)
        pf = plain_fp64(sim, pid_list[0], items[0][1], rtol, args.plain_sample, sig)
        pf["speedup"] = pf["time_to_signal_s_per_pair"] / out["time_to_signal_s_per_pair"]
        out["plain_fp64"] = pf
    sim.close()
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
