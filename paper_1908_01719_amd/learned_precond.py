"""Training driver of the learned polynomial preconditioner (argument
marshalling only).

The interval network (option "precond" = 1) is trained on samples that the
library records from its own Jacobi-CG runs: per system and time step, the
operator's scale features and the extreme Ritz values of that step's CG
coefficients. Recording, gradients and Adam steps run in libdmri's kernels;
this module allocates the device sample buffers with PyTorch and calls the
entry points.

Typical use::

    sim = Simulator(0); sim.set_sequence(seq); pid = sim.add_problem(prob)
    X, T = record(sim, [(pid, b, q)], capacity=1 << 16)   # Jacobi CG runs
    sim.dmri_precond_set_params(learned_guess.init_params(0))
    train(sim, X, T, iters=2000, lr=3e-3)
    sim.set_options(precond=1, cheb_terms=4)              # flexible CG from now on
"""

from __future__ import annotations

from typing import Iterable, Tuple

import numpy as np

from .binding import GUESS_N_FEATURES


def record(sim, runs: Iterable[Tuple[int, np.ndarray, np.ndarray]], capacity: int,
           device: int = 0):
    """Run each (problem_id, b, q) batch with Jacobi CG and the recorder on;
    returns the recorded (features [n, 16], targets [n, 2]) CUDA tensors."""
    import torch
    X = torch.zeros((capacity, GUESS_N_FEATURES), dtype=torch.float32,
                    device="cuda:%d" % device)
    T = torch.zeros((capacity, 2), dtype=torch.float32, device="cuda:%d" % device)
    torch.cuda.synchronize(device)
    pc = sim.dmri_get_option("precond")
    sim.set_options(precond=0)
    sim.dmri_precond_record(X, T, capacity)
    try:
        for pid, b, q in runs:
            b = np.atleast_1d(np.asarray(b, np.float64))
            sim.dmri_run([pid] * len(b), b, q)
    finally:
        n = sim.dmri_precond_record_count()
        sim.dmri_precond_record(None, None, 0)
        sim.set_options(precond=int(pc))
    return X[:n], T[:n]


def train(sim, X, T, iters: int, lr: float, chunk: int = 200):
    """Full-batch Adam on the recorded samples; returns the loss before each
    chunk of iterations and before the last step."""
    hist = []
    done = 0
    last = float("nan")
    while done < iters:
        k = min(chunk, iters - done)
        l0, last = sim.dmri_precond_train(X, T, k, lr)
        hist.append(l0)
        done += k
    hist.append(last)
    return hist


def study(n_train: int = 64, n_eval: int = 128, iters: int = 2000, rtol: float = 1e-8,
          terms=(2, 4, 6), log=print):
    """On the 57^3 cylinder workload: record Jacobi-CG samples of n_train of
    its 1024 systems, train the interval network, then solve n_eval other
    systems (all FP64, damped cubic guess) with Jacobi CG, with the reference
    interval [0.5, 1.5] and with the learned interval for each number of
    terms. Returns iterations, operator products and solve times per run and
    the signals' largest deviation from Jacobi CG's."""
    import time

    import torch

    import dmri_inputs as di

    from .binding import Simulator
    from .learned_guess import init_params, zero_params

    torch.zeros(1, device="cuda")
    prob, seq, sl = di.cylinder_57_batched()
    n_all = len(sl.b)
    pick = np.linspace(0, n_all - 1, n_train).round().astype(int)
    rest = np.setdiff1d(np.arange(n_all), pick)
    ev = rest[np.linspace(0, len(rest) - 1, n_eval).round().astype(int)]
    out = {"workload": "cylinder_57_batched", "rtol": rtol, "n_train": n_train,
           "n_eval": n_eval, "runs": {}}
    with Simulator(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(precision=0, rtol=rtol, guess=1)
        pid = sim.add_problem(prob)
        t0 = time.perf_counter()
        X, T = record(sim, [(pid, sl.b[pick], sl.q[pick])], capacity=n_train * 240)
        out["samples"] = int(X.shape[0])
        out["record_s"] = time.perf_counter() - t0
        sim.dmri_precond_set_params(zero_params())
        out["loss_zero"], _ = sim.dmri_precond_train(X, T, 1, 1e-12)
        sim.dmri_precond_set_params(init_params(0))
        t0 = time.perf_counter()
        hist = train(sim, X, T, iters=iters, lr=3e-3)
        out["loss"] = [float(hist[0]), float(hist[-1])]
        out["train_s"] = time.perf_counter() - t0
        log("recorded %d samples in %.1fs; loss %.3e -> %.3e (zero network %.3e) in %.1fs" % (
            out["samples"], out["record_s"], hist[0], hist[-1], out["loss_zero"],
            out["train_s"]))
        b, q = sl.b[ev], sl.q[ev]
        cases = [("jacobi", dict(precond=0), 1), ("reference_interval_4",
                                                   dict(precond=2, cheb_terms=4), 4)]
        cases += [("learned_%d" % m, dict(precond=1, cheb_terms=m), m) for m in terms]
        sigs = {}
        for name, opts, m in cases:
            sim.set_options(**opts)
            sig, st = sim.dmri_run([pid] * len(b), b, q)
            per = st["total_iterations"] / (len(b) * 240.0)
            out["runs"][name] = {"solve_s": st["t_solve_s"], "iterations_per_system_step": per,
                                 "operator_products_per_system_step": per * m,
                                 "fallback_steps": sim.dmri_get_option("pc_fallback_steps")}
            sigs[name] = sig
            log("%s: %s" % (name, json_line(out["runs"][name])))
        for name in sigs:
            out["runs"][name]["max_rel_dev_vs_jacobi"] = float(
                np.max(np.abs(sigs[name] - sigs["jacobi"]) / np.abs(sigs["jacobi"])))
        sim.set_options(precond=0)
    return out


def json_line(d) -> str:
    import json
    return json.dumps(d, sort_keys=True)


if __name__ == "__main__":
    import argparse
    import sys

    ap = argparse.ArgumentParser(description="study of the learned polynomial preconditioner")
    ap.add_argument("--n-train", type=int, default=64)
    ap.add_argument("--n-eval", type=int, default=128)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--rtol", type=float, default=1e-8)
    a = ap.parse_args()
    res = study(n_train=a.n_train, n_eval=a.n_eval, iters=a.iters, rtol=a.rtol,
                log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json_line(res))
