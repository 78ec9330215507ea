"""Training driver of the learned initial guess (argument marshalling only).

Samples, gradients and Adam steps all run in libdmri's kernels; this module
allocates the device sample buffers with PyTorch, drives the recorder during
ordinary simulation runs, and calls the training entry points.

Typical use::

    sim = Simulator(0); sim.set_sequence(seq); pid = sim.add_problem(prob)
    X, T = record(sim, [(pid, b, q)], capacity=1 << 20, stride=97)
    sim.dmri_guess_set_params(init_params(0))
    train(sim, X, T, iters=2000, lr=2e-3)
    sim.set_options(guess=2)           # later runs start from the network's guess
"""

from __future__ import annotations

from typing import Iterable, Tuple

import numpy as np

from .binding import GUESS_N_FEATURES, GUESS_N_PARAMS

N_IN, N_HID, N_OUT = GUESS_N_FEATURES, 64, 2


def init_params(seed: int = 0, out_scale: float = 0.1) -> np.ndarray:
    """He-normal hidden layers, a small output layer, zero biases (packed
    W1, b1, W2, b2, W3, b3 as the library expects)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(N_IN, N_HID)) * np.sqrt(2.0 / N_IN)
    W2 = rng.normal(size=(N_HID, N_HID)) * np.sqrt(2.0 / N_HID)
    W3 = rng.normal(size=(N_HID, N_OUT)) * np.sqrt(1.0 / N_HID) * out_scale
    p = np.concatenate([W1.ravel(), np.zeros(N_HID), W2.ravel(), np.zeros(N_HID), W3.ravel(),
                        np.zeros(N_OUT)]).astype(np.float32)
    assert p.size == GUESS_N_PARAMS
    return p


def zero_params() -> np.ndarray:
    """All-zero network: its guess is the damped cubic extrapolation itself."""
    return np.zeros(GUESS_N_PARAMS, np.float32)


def record(sim, runs: Iterable[Tuple[int, np.ndarray, np.ndarray]], capacity: int, stride: int,
           device: int = 0):
    """Run each (problem_id, b, q) batch with the recorder on; returns the
    recorded (features [n, 16], targets [n, 2]) float32 CUDA tensors."""
    import torch
    X = torch.zeros((capacity, N_IN), dtype=torch.float32, device="cuda:%d" % device)
    T = torch.zeros((capacity, 2), dtype=torch.float32, device="cuda:%d" % device)
    torch.cuda.synchronize(device)
    sim.dmri_guess_record(X, T, capacity, stride)
    try:
        for pid, b, q in runs:
            b = np.atleast_1d(np.asarray(b, np.float64))
            sim.dmri_run([pid] * len(b), b, q)
    finally:
        n = sim.dmri_guess_record_count()
        sim.dmri_guess_record(None, None, 0, 1)
    return X[:n], T[:n]


def train(sim, X, T, iters: int, lr: float, chunk: int = 200):
    """Full-batch Adam on the recorded samples; returns the loss history
    (one value per chunk of iterations, then the final loss)."""
    hist = []
    done = 0
    while done < iters:
        k = min(chunk, iters - done)
        l0, _ = sim.dmri_guess_train(X, T, k, lr)
        hist.append(l0)
        done += k
    hist.append(sim.dmri_guess_eval(X, T))
    return hist


def held_out_study(n_train_sys: int = 64, iters: int = 2000, seeds=(100, 101, 102, 103),
                   n_held: int = 78, precision: int = 1, rtol: float = 1e-6, log=print):
    """Train on solver trajectories of the 57^3 cylinder workload (a spread
    of n_train_sys of its 1024 systems) and of the eight seeded-cell
    geometries (32 pairs each), then run held-out seeded geometries at
    n_held cubes per side with the previous-step guess, the damped cubic
    extrapolation and the learned correction. Returns a dict of the Krylov
    iterations per system and step, solve times and signal deviations."""
    import time

    import torch

    import dmri_inputs as di

    from .binding import Simulator

    # the sample buffers are PyTorch tensors: bring up its device context first
    torch.zeros(1, device="cuda")
    out = {"train": {}, "held_out": []}
    with Simulator(0) as sim:
        sim.set_sequence(di.PGSE_SHORT)
        sim.set_options(precision=precision, rtol=rtol, guess=1)
        runs = []
        prob, _, sl = di.cylinder_57_batched()
        pick = np.linspace(0, len(sl) - 1, n_train_sys).round().astype(int)
        runs.append((sim.add_problem(prob), sl.b[pick], sl.q[pick]))
        for seed in range(8):
            p, _, s8 = di.seeded_cells(seed)
            runs.append((sim.add_problem(p), s8.b, s8.q))
        t0 = time.perf_counter()
        X, T = record(sim, runs, capacity=1_500_000, stride=997)
        out["train"]["samples"] = int(X.shape[0])
        out["train"]["record_s"] = time.perf_counter() - t0
        log("recorded %d samples in %.1fs" % (X.shape[0], out["train"]["record_s"]))
        sim.dmri_guess_set_params(zero_params())
        out["train"]["loss_zero"] = sim.dmri_guess_eval(X, T)
        sim.dmri_guess_set_params(init_params(0))
        t0 = time.perf_counter()
        hist = train(sim, X, T, iters=iters, lr=2e-3)
        out["train"]["loss"] = [float(v) for v in (hist[0], hist[-1])]
        out["train"]["train_s"] = time.perf_counter() - t0
        log("trained: loss %.3e -> %.3e (zero network %.3e) in %.1fs"
            % (hist[0], hist[-1], out["train"]["loss_zero"], out["train"]["train_s"]))
        for seed in seeds:
            p, _, s8 = di.seeded_cells(seed, n_fixed=n_held)
            pid = sim.add_problem(p)
            Xv, Tv = record(sim, [(pid, s8.b[:4], s8.q[:4])], capacity=200_000, stride=101)
            rec = {"seed": seed, "n_dof": sim.dmri_problem_info(pid)[0],
                   "loss_trained": sim.dmri_guess_eval(Xv, Tv)}
            theta = sim.dmri_guess_get_params()
            sim.dmri_guess_set_params(zero_params())
            rec["loss_zero"] = sim.dmri_guess_eval(Xv, Tv)
            sim.dmri_guess_set_params(theta)
            sigs = {}
            for g in (0, 1, 2):
                sim.set_options(guess=g)
                sig, st = sim.dmri_run([pid] * len(s8.b), s8.b, s8.q)
                n_steps = 240
                rec["guess%d" % g] = {
                    "iterations_per_system_step": st["total_iterations"] / (len(s8.b) * n_steps),
                    "solve_s": st["t_solve_s"],
                    "time_to_signal_s": st["t_solve_s"] / len(s8.b)}
                sigs[g] = sig
            rec["max_rel_dev_vs_damped_cubic"] = {
                str(g): float(np.max(np.abs(sigs[g] - sigs[1]) / np.abs(sigs[1]))) for g in (0, 2)}
            log(json_line(rec))
            out["held_out"].append(rec)
        sim.set_options(guess=1)
    return out


def json_line(d) -> str:
    import json
    return json.dumps(d, sort_keys=True)


if __name__ == "__main__":
    import argparse
    import sys

    ap = argparse.ArgumentParser(description="held-out study of the learned guess")
    ap.add_argument("--n-held", type=int, default=78)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--seeds", type=int, nargs="*", default=[100, 101, 102, 103])
    a = ap.parse_args()
    res = held_out_study(iters=a.iters, seeds=tuple(a.seeds), n_held=a.n_held,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json_line(res))
