"""The conventional AIM operator of Sec. II-B, beside AIMx (oracle).

    A(k) x  ~=  A_NR(k) x  -  A_P(k) x  +  W H(k) P x        (eqs. aimL, aimLFR)

* A_NR(k) holds the near-region Galerkin entries of the full kernel
  G(k, R) = e^{-jkR}/(4 pi R) by direct integration.  Reading (the paper
  leaves the singular integration to standard techniques): the singular
  static part G_s is integrated as in AIMx (closed-form inner integral,
  3-point outer rule, symmetrised: the A_s,NR of the AIMx oracle) and the
  smooth remainder G_d = G - G_s (eq. hgfd, -jk/(4 pi) at R = 0 by
  eq. hgfdtaylor) by the 3 x 3 point rule, the same split the dense
  reference uses.
* A_P(k) = W H_NR(k) P (eq. aimLP): H_NR has the entries of H(k) for the
  grid points of near pairs, G(k, h|d|) off the diagonal and on it the self
  term of the far-field H (-jk/(4 pi), eq. Hmm).  The paper notes that in the
  conventional AIM the self term may take any value as long as H and H_NR
  share it; with the shared value it cancels.
* W H(k) P is the far operator of AIMx unchanged (same grid, stencils and
  kernel spectrum).

Per wavenumber the complex correction C(k) = A_NR(k) - A_P(k) must be
rebuilt; AIMx replaces it by one real, frequency-independent C (Sec. III-A),
which is the saving the paper measures over frequency sweeps (Sec. VI).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mesh as _mesh
from .aimx import AimOracle, static_near
from .green import FOUR_PI, green_dynamic, green_full


def dynamic_near(V, T, rows, cols, k: float) -> np.ndarray:
    """Entries of the smooth part of A_NR(k) on the given pairs:
    sum_p sum_q (A_i/3)(A_j/3) G_d(k, |r_ip - r_jq|), the 3 x 3 point rule."""
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    d = qp[rows][:, :, None, :] - qp[cols][:, None, :, :]     # [pairs, p, q, xyz]
    R = np.linalg.norm(d, axis=-1)
    ww = w[rows][:, :, None] * w[cols][:, None, :]
    return np.sum(ww * green_dynamic(k, R), axis=(1, 2))


def precorrection_with(Pm: sp.csr_matrix, rows, cols, dims, h: float, kernel) -> np.ndarray:
    """sum_u sum_v P[u,i] K(r_u - r_v) P[v,j] on the given pairs, for a grid
    kernel given as a function of the distance array (whose zero entries
    must map to the self term)."""
    Pc = Pm.tocsc()
    Nx, Ny, _ = dims
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty(rows.size, dtype=np.complex128)

    def column(j):
        sl = slice(Pc.indptr[j], Pc.indptr[j + 1])
        u = Pc.indices[sl]
        xyz = np.stack([u % Nx, (u // Nx) % Ny, u // (Nx * Ny)], axis=1).astype(np.float64)
        return xyz, Pc.data[sl]

    for t, (i, j) in enumerate(zip(rows, cols)):
        xi, wi = column(int(i))
        xj, wj = column(int(j))
        R = h * np.linalg.norm(xi[:, None, :] - xj[None, :, :], axis=-1)
        out[t] = wi @ kernel(R) @ wj
    return out


def full_grid_kernel(k: float):
    """The grid kernel of H(k): G(k, R) for R > 0 and -jk/(4 pi) at R = 0."""
    def kern(R):
        R = np.asarray(R, dtype=np.float64)
        out = np.empty(R.shape, dtype=np.complex128)
        nz = R > 0
        out[nz] = green_full(k, R[nz])
        out[~nz] = -1j * k / FOUR_PI
        return out
    return kern


class ConventionalAim:
    """Conventional AIM on the same mesh, grid and far operator as an
    AimOracle."""

    def __init__(self, aim: AimOracle):
        self.o = aim
        self._C = {}

    def correction_values(self, rows, cols, k: float) -> np.ndarray:
        """C(k) = A_NR(k) - A_P(k) on the given pairs."""
        o = self.o
        anr = static_near(o.V, o.T, rows, cols) + dynamic_near(o.V, o.T, rows, cols, k)
        ap = precorrection_with(o.P, rows, cols, o.dims, o.h, full_grid_kernel(k))
        return anr - ap

    def correction(self, k: float) -> sp.csr_matrix:
        """The whole complex near correction (small problems only)."""
        key = float(k)
        if key not in self._C:
            rows, cols = self.o.near_list()
            vals = self.correction_values(rows, cols, key)
            self._C[key] = sp.csr_matrix((vals, (rows, cols)), shape=(self.o.N, self.o.N))
        return self._C[key]

    def matvec(self, x, k: float) -> np.ndarray:
        """y = A_NR(k) x - A_P(k) x + W H(k) P x."""
        x = np.asarray(x, dtype=np.complex128)
        y = self.o.far(x, k)
        C = self.correction(k)
        if x.ndim == 1:
            return y + C @ x
        return y + (C @ x.T).T
