"""Right-hand sides: Galerkin-tested incident fields (oracle).

b_i = sum_p (A_i/3) u_inc(r_ip) with the 3-point rule of ``mesh``.

* plane wave travelling along +z with the e^{j omega t} convention
  (Sec. II): u_inc(r) = exp(-j k z);
* Gaussian patch of width sigma about a centre p:
  u_inc(r) = exp(-|r - p|^2 / (2 sigma^2)).
"""
from __future__ import annotations

import numpy as np

from . import mesh as _mesh


def plane_wave(V, T, k: float, direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    return np.sum(w * np.exp(-1j * k * (qp @ d)), axis=1)


def gaussian_patch(V, T, centre, sigma: float) -> np.ndarray:
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    r2 = np.sum((qp - np.asarray(centre, dtype=np.float64)) ** 2, axis=-1)
    return np.sum(w * np.exp(-r2 / (2.0 * sigma * sigma)), axis=1).astype(np.complex128)
