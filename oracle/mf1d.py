"""Matrix-formalism reference signal for a 1-D slab (oracle pin, FP64).

Test infrastructure only (see the package header).

The paper validates its signals against matrix-formalism (MF) references
(Sec. 4). For an interval [-L/2, L/2] with reflecting walls the Laplacian
eigenfunctions are known in closed form,
  phi_0 = 1/sqrt(L),  phi_m = sqrt(2/L) cos(m pi (x + L/2) / L),
  lambda_m = D (m pi / L)^2,
so expanding U(x,t) = sum_m c_m(t) phi_m(x) turns the Bloch-Torrey
equation (Sec. 2, eq. strong_BT) with g along x into the ODE system
  c' = -(Lambda + i G f(t) X + 1/T2) c,   X_mn = int x phi_m phi_n dx,
which is integrated exactly with matrix exponentials over the pieces where
f is constant. The signal is S = int U(T) = sqrt(L) c_0(T).

The expansion is truncated to n_modes; its convergence in n_modes is part
of the pin test.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _basis(L, n_modes, xq):
    m = np.arange(n_modes)[:, None]
    phi = np.sqrt(2.0 / L) * np.cos(m * np.pi * (xq[None, :] + 0.5 * L) / L)
    phi[0, :] = 1.0 / np.sqrt(L)
    return phi


def slab_signal(L, D, G, delta, Delta, T2=None, n_modes=64, n_quad=4096):
    """Signal per unit cross-section of a PGSE experiment in a slab of width L.

    G = gamma |g| in rad/(um us), gradient along the slab normal, uniform
    initial magnetization 1, echo at T = Delta + delta.
    """
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    x = 0.5 * L * xg
    w = 0.5 * L * wg
    phi = _basis(L, n_modes, x)
    X = (phi * (w * x)[None, :]) @ phi.T
    lam = D * (np.arange(n_modes) * np.pi / L) ** 2
    r2 = 0.0 if T2 is None else 1.0 / T2
    Lam = np.diag(lam + r2)
    c = np.zeros(n_modes, dtype=np.complex128)
    c[0] = np.sqrt(L)
    pieces = [(+1.0, delta), (0.0, Delta - delta), (-1.0, delta)]
    for f, tau in pieces:
        if tau <= 0:
            continue
        c = sla.expm(-(Lam + 1j * G * f * X) * tau) @ c
    return np.sqrt(L) * c[0]
