"""The magnetic-field (double-layer) operator on RWG functions under AIMx
(oracle; test infrastructure only, used by tests/ and nothing in the
library).

Sec. III-B (eqs. opK, ghgf, opKs, opKd, KAIMx, gH00) with RWG functions
f_n and Galerkin testing (the discrete CFIE, eq. CFIEdis, tests n x n x K
with the RWG functions, i.e. f_m . (n x K[f_n]) for tangential f_m):

    K_mn = int f_m(r) . [ n(r) x int grad G(r, r') x f_n(r') dS' ] dS,
    grad G = -(r - r') (1 + jkR) e^{-jkR} / (4 pi R^3)     (eq. ghgf),

with n the unit normal (b - a) x (c - a) of the testing triangle, in the
principal-value sense: on a flat testing triangle's own points r - r' and
f_n both lie in its plane, so the integrand is normal and n x it vanishes.
The residue of the surface limit (the +-J/2 of the MFIE) is a multiple of
the Gram matrix G_mn = int f_m . f_n dS, kept separately here; the library
applies K + beta G.

AIMx (eq. KAIMx):  K ~= K_s,NR - K_s,P + W H_grad(k) P.

* K_s,NR: the static kernel grad G_s = -(r - r')/(4 pi R^3) (eq. ghgfs) on
  the RWG near list.  With f_n = s l/(2A) (r' - p) on its triangle T and
  (r - r') x (r' - r) = 0,
      int_T grad G_s x f_n dS' = -(s l/(2A)) (1/4 pi) g(r) x (r - p),
      g(r) = int_T (r - r')/R^3 dS' = sum_i m_i int_{edge i} dl/R + n_T sign(h) Omega,
  m_i the outward in-plane edge normals, h the height of r above T and
  Omega the solid angle T subtends at r (the in-plane part is the gradient
  theorem for grad_s' (1/R); the normal part is the solid angle); 3-point
  outer rule.  In the plane of T (h = 0) the normal part is its principal
  value, 0.
* P: three current channels, the projections of w_q f_n(r_q) at the
  quadrature points (those of the EFIE); W: the projections of
  w_q f_m(r_q) x n at the same points (so that the tested value is
  W^T V with V the grid field).
* H_grad: the grid samples of grad G(r_u - r_v), 0 at u = v (reading: eq.
  gH00 gives a scalar for this vector kernel; 0 per component is the
  symmetric value).  The grid field V(u) = sum_v H_grad(u - v) x J(v) is
  evaluated as the plain definition: component a = H_b * J_c - H_c * J_b,
  six zero-padded circulant convolutions.
* K_s,P = W H_grad,s P on the near list with the static samples.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import mesh as _mesh
from .aimx import AimOracle, grid_convolve
from .dlp import circulant_grad_kernels, grad_kernel
from .efie import EfieOracle, Rwg, channel_projections
from .green import FOUR_PI


# --------------------------------------------------------------------------
# closed form of the static gradient integral
# --------------------------------------------------------------------------

def triangle_grad_inv_r(r, a, b, c) -> np.ndarray:
    """int_T (r - r') / |r - r'|^3 dS' (vector) in closed form; the normal
    part is 0 for r in the plane of T (principal value)."""
    r = np.asarray(r, dtype=np.float64)
    v = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(v[1] - v[0], v[2] - v[0])
    size = math.sqrt(np.linalg.norm(n))
    n = n / np.linalg.norm(n)
    h = float(np.dot(r - v[0], n))
    out = np.zeros(3)
    for i in range(3):
        p, q = v[i], v[(i + 1) % 3]
        L = float(np.linalg.norm(q - p))
        t = (q - p) / L
        m = np.cross(t, n)
        P0 = float(np.dot(p - r, m))
        lm = float(np.dot(p - r, t))
        lp = float(np.dot(q - r, t))
        Rm = float(np.linalg.norm(p - r))
        Rp = float(np.linalg.norm(q - r))
        R0sq = P0 * P0 + h * h
        # int_{lm}^{lp} dl / sqrt(l^2 + R0^2), free of cancellation
        if lm >= 0.0:
            f = math.log((Rp + lp) / (Rm + lm))
        elif lp <= 0.0:
            f = math.log((Rm - lm) / (Rp - lp))
        else:
            f = math.log((Rp + lp) * (Rm - lm) / R0sq)
        out = out + m * f
    if abs(h) > 1e-14 * size:
        A, B, C = v[0] - r, v[1] - r, v[2] - r
        la, lb, lc = np.linalg.norm(A), np.linalg.norm(B), np.linalg.norm(C)
        num = abs(float(np.dot(A, np.cross(B, C))))
        den = la * lb * lc + np.dot(A, B) * lc + np.dot(A, C) * lb + np.dot(B, C) * la
        omega = 2.0 * math.atan2(num, den)
        out = out + n * math.copysign(omega, h)
    return out


def triangle_grad_inv_r_quadrature(r, a, b, c, order: int = 80) -> np.ndarray:
    """The same integral by Gauss-Legendre quadrature over the triangle
    (Duffy map from vertex a); for points off the triangle only."""
    r = np.asarray(r, dtype=np.float64)
    A, B, C = (np.asarray(x, float) for x in (a, b, c))
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    U, Vv = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    two_area = float(np.linalg.norm(np.cross(B - A, C - A)))
    pts = A[None, None, :] + U[..., None] * (B - A)[None, None, :] \
        + (U * Vv)[..., None] * (C - B)[None, None, :]
    d = r[None, None, :] - pts
    R = np.linalg.norm(d, axis=-1)
    return two_area * np.einsum("ij,ijk->k", W * U / R ** 3, d)


# --------------------------------------------------------------------------
# the operator
# --------------------------------------------------------------------------

def testing_values(rwg: Rwg) -> np.ndarray:
    """w_q f(r_q) x n for every triangle, point and local edge: [N, 3, 3, 3]."""
    vals = rwg.point_values()[..., :3]
    nrm = _mesh.unit_normals(rwg.V, rwg.T)
    return np.cross(vals, nrm[:, None, None, :])


class MfieOracle:
    """K and the Gram matrix G on the RWG functions, grid, stencils and
    near list of an EfieOracle."""

    def __init__(self, e: EfieOracle):
        self.e = e
        self.o = e.o
        self.rwg = e.rwg
        self.n = e.n
        self.J = e.P[:3]                                   # current channels
        self.Wt = channel_projections(self.rwg, self.o, testing_values(self.rwg))
        self.rows, self.cols = e.rows, e.cols
        self._tris = {}
        for t in range(self.rwg.T.shape[0]):
            for ed in range(3):
                m = self.rwg.tri_rwg[t, ed]
                if m >= 0:
                    self._tris.setdefault(int(m), []).append((t, ed))
        self._qp = _mesh.quad_points(self.rwg.V, self.rwg.T)
        self._tv = testing_values(self.rwg)
        self._g = {}

    def _grad(self, tm: int, tn: int):
        """g(r_q) = int_{T_tn} (r_q - r')/R^3 at the three points of tm."""
        key = (tm, tn)
        if key not in self._g:
            V, T = self.rwg.V, self.rwg.T
            a, b, c = (V[T[tn, i]] for i in range(3))
            self._g[key] = np.array([triangle_grad_inv_r(self._qp[tm, q], a, b, c)
                                     for q in range(3)])
        return self._g[key]

    def static_entry(self, m: int, n: int) -> float:
        rwg = self.rwg
        acc = 0.0
        for tm, em in self._tris[m]:
            tv = self._tv[tm, :, em, :]                     # [3, 3]
            for tn, en in self._tris[n]:
                g = self._grad(tm, tn)
                coef = rwg.tri_sign[tn, en] * rwg.length[n] / (2.0 * rwg.area[tn])
                p = rwg.V[rwg.T[tn, en]]
                inner = -coef / FOUR_PI * np.cross(g, self._qp[tm] - p[None, :])
                acc += float(np.sum(tv * inner))
        return acc

    def static_near(self, rows, cols) -> np.ndarray:
        return np.array([self.static_entry(int(m), int(n)) for m, n in zip(rows, cols)])

    def precorrection(self, rows, cols) -> np.ndarray:
        """sum_u sum_v W(u) . (H_grad,s(u - v) x J(v)) on the given pairs."""
        o = self.o
        Nx, Ny, _ = o.dims
        kern = grad_kernel(0.0, o.h, True)                  # = -grad G_s on the grid
        if not hasattr(self, "_csc"):
            self._csc = ([w.tocsc() for w in self.Wt], [j.tocsc() for j in self.J], {}, {})
        Wc, Jc, wcache, jcache = self._csc

        def nodes(mats, j, cache):
            if j not in cache:
                parts = [(m.indices[m.indptr[j]:m.indptr[j + 1]], m.data[m.indptr[j]:m.indptr[j + 1]])
                         for m in mats]
                idx = np.unique(np.concatenate([ii for ii, _ in parts]))
                vals = np.zeros((idx.size, len(mats)))
                for c, (ii, dd) in enumerate(parts):
                    vals[np.searchsorted(idx, ii), c] = dd
                xyz = np.stack([idx % Nx, (idx // Nx) % Ny, idx // (Nx * Ny)], axis=1)
                cache[j] = (xyz.astype(np.float64), vals)
            return cache[j]

        out = np.empty(len(rows))
        for t, (m, n) in enumerate(zip(rows, cols)):
            xm, wm = nodes(Wc, int(m), wcache)
            xn, jn = nodes(Jc, int(n), jcache)
            H = -kern(xm[:, None, :] - xn[None, :, :]).real  # grad G_s samples
            Vf = np.cross(H, jn[None, :, :]).sum(axis=1)       # [nm, 3]
            out[t] = float(np.sum(wm * Vf))
        return out

    def correction_values(self, rows, cols) -> np.ndarray:
        """C_K = K_s,NR - K_s,P on the given RWG pairs."""
        return self.static_near(rows, cols) - self.precorrection(rows, cols)

    def gram(self, rows, cols) -> np.ndarray:
        """G_mn = int f_m . f_n (3-point rule, exact for the quadratic integrand)."""
        vals = self.rwg.point_values()[..., :3]
        w = _mesh.quad_weights(self.rwg.V, self.rwg.T)
        out = np.zeros(len(rows))
        for t, (m, n) in enumerate(zip(rows, cols)):
            for tm, em in self._tris[int(m)]:
                for tn, en in self._tris[int(n)]:
                    if tm == tn:
                        out[t] += float(np.sum(vals[tm, :, em, :] * vals[tm, :, en, :]
                                               / w[tm][:, None]))
        return out

    def far(self, x, k: float) -> np.ndarray:
        o = self.o
        Nx, Ny, Nz = o.dims
        S = np.fft.fftn(circulant_grad_kernels(k, o.dims, o.h), axes=(-3, -2, -1))
        Jg = [(self.J[c] @ x).reshape(Nz, Ny, Nx) for c in range(3)]
        y = 0.0
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            # grad G = -kern: V_a = -(K_b * J_c - K_c * J_b)
            Va = -(grid_convolve(Jg[c], S[b], o.dims) - grid_convolve(Jg[b], S[c], o.dims))
            y = y + self.Wt[a].T @ Va.reshape(-1)
        return y

    def matvec_rows(self, x, k: float, rows, beta: float = 0.0) -> np.ndarray:
        """Selected entries of (K + beta G) x."""
        rows = np.unique(np.asarray(rows, dtype=np.int64))
        sel = np.isin(self.rows, rows)
        r, c = self.rows[sel], self.cols[sel]
        v = self.correction_values(r, c) + beta * self.gram(r, c)
        Cs = sp.csr_matrix((v, (r, c)), shape=(self.n, self.n))
        x = np.asarray(x, dtype=np.complex128)
        return self.far(x, k)[rows] + (Cs @ x)[rows]

    def matvec(self, x, k: float, beta: float = 0.0) -> np.ndarray:
        return self.matvec_rows(x, k, np.arange(self.n), beta)


def dense_rows(rwg: Rwg, k: float, rows, mo: MfieOracle | None = None) -> np.ndarray:
    """Rows of the dense K by direct integration: the static kernel in
    closed form, the smooth remainder grad G_d = grad G - grad G_s by the
    3 x 3 point rule (0 at R = 0, its limit's symmetric value)."""
    rows = np.asarray(rows, dtype=np.int64)
    n_all = rwg.n
    if mo is None:
        raise ValueError("needs an MfieOracle for the static entries")
    out = np.zeros((rows.size, n_all), dtype=np.complex128)
    V, T = rwg.V, rwg.T
    qp = _mesh.quad_points(V, T)
    vals = rwg.point_values()[..., :3]
    tv = testing_values(rwg)
    for a, m in enumerate(rows):
        for n in range(n_all):
            acc = mo.static_entry(int(m), n)
            for tm, em in mo._tris[int(m)]:
                for tn, en in mo._tris[n]:
                    d = qp[tm][:, None, :] - qp[tn][None, :, :]      # r - r'
                    R = np.linalg.norm(d, axis=-1)
                    with np.errstate(divide="ignore", invalid="ignore"):
                        f = np.where(R > 0, -((1 + 1j * k * R) * np.exp(-1j * k * R) - 1.0)
                                     / (FOUR_PI * np.where(R > 0, R, 1.0) ** 3), 0.0)
                    gd = d * f[..., None]                              # grad G_d
                    cr = np.cross(gd, vals[tn, None, :, en, :])        # [3, 3, 3]
                    acc += np.sum(tv[tm, :, em, None, :] * cr)
            out[a, n] = acc
    return out
