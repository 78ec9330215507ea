"""Pin of the NumPy MLP reference: chain-rule gradients vs central finite
differences of the loss, on random inputs (no kinks hit: |z| bounded away
from 0 is checked)."""

import numpy as np

from oracle import mlp


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    theta = mlp.init(seed=1)
    x = rng.normal(size=(20, mlp.N_IN))
    t = rng.normal(size=(20, mlp.N_OUT))
    g = mlp.gradients(theta, x, t)
    assert g.shape == (mlp.n_params(),) == (5378,)
    idx = rng.choice(mlp.n_params(), size=60, replace=False)
    eps = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss(tp, x, t) - mlp.loss(tm, x, t)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_shapes_and_pack_roundtrip():
    theta = mlp.init(seed=2)
    parts = mlp.unpack(theta)
    assert np.array_equal(mlp.pack(parts), theta)
    y, _ = mlp.forward(theta, np.zeros((3, mlp.N_IN)))
    assert y.shape == (3, 2)
