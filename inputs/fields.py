"""Nodal values of the synthetic source fields (evaluation only, no assembly).

* The manufactured solution u = cos(pi x) cos(pi y) sin(pi z / (2H)) on the
  box [0,1]^2 x [-H, 0] vanishes on the top surface and has zero normal
  derivative on the floor and on the vertical coasts; its source is
  f = -Lap u = (2 pi^2 + pi^2 / (4 H^2)) u.
* The smooth random field is a sum of 16 Fourier modes with N(0,1)
  amplitudes drawn from ``np.random.default_rng(seed).standard_normal(16)``:
  cos(k pi x) cos(l pi y) for (k, l) in {0..3}^2 without (0, 0), in row-major
  (k, l) order, followed by cos(pi z / H).
"""
from __future__ import annotations

import numpy as np


def manufactured_u(xyz: np.ndarray, H: float) -> np.ndarray:
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.cos(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * z / (2.0 * H))


def manufactured_f(xyz: np.ndarray, H: float) -> np.ndarray:
    return (2.0 * np.pi ** 2 + np.pi ** 2 / (4.0 * H * H)) * manufactured_u(xyz, H)


def fourier_field(xyz: np.ndarray, H: float, seed: int) -> np.ndarray:
    a = np.random.default_rng(seed).standard_normal(16)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    f = np.zeros(xyz.shape[0])
    m = 0
    for k in range(4):
        for l in range(4):
            if k == 0 and l == 0:
                continue
            f += a[m] * np.cos(k * np.pi * x) * np.cos(l * np.pi * y)
            m += 1
    f += a[15] * np.cos(np.pi * z / H)
    return f
