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
