"""NumPy reference of the learned-initial-guess network (oracle, FP64).

Test infrastructure only (see the package header).

The network is a per-sample multilayer perceptron
    h1 = relu(x W1 + b1),  h2 = relu(h1 W2 + b2),  y = h2 W3 + b3
with x of 16 features, 64 hidden units per layer and 2 outputs, trained with
the mean squared error L = sum((y - t)^2) / n over a batch of n samples.
`forward` and `gradients` are the plain definitions (matrix products and the
chain rule); the tests pin `gradients` against central finite differences of
`loss`, and the GPU kernels (BF16 operands, FP32 accumulation) against both.

Parameter order (also the packed order of the library's weight blob):
W1 [16, 64], b1 [64], W2 [64, 64], b2 [64], W3 [64, 2], b3 [2].
"""

from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 16, 64, 2
SHAPES = [(N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_OUT), (N_OUT,)]


def n_params() -> int:
    return int(sum(np.prod(s) for s in SHAPES))


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def init(seed=0, scale=1.0):
    """He-style random initial parameters (packed)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(N_IN, N_HID)) * np.sqrt(2.0 / N_IN) * scale
    W2 = rng.normal(size=(N_HID, N_HID)) * np.sqrt(2.0 / N_HID) * scale
    W3 = rng.normal(size=(N_HID, N_OUT)) * np.sqrt(1.0 / N_HID) * scale
    return pack([W1, np.zeros(N_HID), W2, np.zeros(N_HID), W3, np.zeros(N_OUT)])


def forward(theta, x):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(theta, x, t):
    y, _ = forward(theta, x)
    return float(np.sum((y - t) ** 2) / x.shape[0])


def gradients(theta, x, t):
    """dL/dtheta (packed) by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (x, z1, h1, z2, h2) = forward(theta, x)
    n = x.shape[0]
    dy = 2.0 * (y - t) / n
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])
