"""The double-layer potential operator under AIMx (oracle; test
infrastructure only, used by tests/, smoke() and the bench's CPU baseline).

Sec. III-B (eqs. opK, ghgf, ghgftaylor, opKs, opKd, Kmatdecomp, KAIMx,
gH00) applies AIMx to the double-layer operator, whose kernel is the
gradient of G (eq. ghgf; the gradient with respect to the observation
point r, with unit vector r^ = (r - r')/R).  This build keeps the scalar
setting of the single-layer path: one piecewise-constant density per flat
triangle, Galerkin testing, and the scalar double-layer kernel

    dG/dn' = n_j . grad' G(r, r') = n_j . (r - r') (1 + jkR) e^{-jkR} / (4 pi R^3)

(grad' = -grad), so that

    (K x)_i = sum_j x_j  int_{T_i} int_{T_j} dG/dn'(r, r') dS' dS.

Self pairs are taken in the principal-value sense: the observation point
lies in the plane of its own flat triangle, where n_j . (r - r') = 0, so the
self entries vanish; the jump term (+-x/2 on a closed surface) is a separate
identity term the caller adds (the paper's analytical residue term).

AIMx (eq. KAIMx):  K(k) ~= K_s,NR - K_s,P + W H_grad(k) P^(K).

* K_s,NR: the static kernel n_j.(r - r')/(4 pi R^3) (the singular first term
  of eq. ghgftaylor) on near pairs, inner integral in closed form: for r at
  signed height h above the plane of T, int_T h / R^3 dS' = sign(h) times the
  solid angle of T seen from r, which is the arctangent sum of the edge-sum
  formula for the 1/R potential (oracle.potential) -- derived here from
  d/dh of that formula; outer integral by the 3-point rule.
* P^(K): three channels, a = x, y, z: P diag(n_a) (the source's dipole
  direction times its projection).
* H_grad: per channel, the grid samples of dG/dr'_a between nodes u and v,
  h (u_a - v_a) (1 + jkR) e^{-jkR} / (4 pi R^3) with R = h |u - v| (odd in
  u_a - v_a, even in the other axes).  Reading: eq. gH00 gives a scalar self
  term for this vector kernel, whose direction is undefined at R = 0; the
  symmetric value, 0 per component, is used (the odd kernel's own value).
* K_s,P = W H_grad,s,NR P^(K) on near pairs with the static samples
  h (u_a - v_a) / (4 pi R^3).
* W = P^T (Galerkin testing).

The far product is evaluated here as the plain definition: three
zero-padded circulant FFT convolutions with the odd kernels, summed.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.sparse as sp

from . import mesh as _mesh
from .aimx import AimOracle, FFT_WORKERS, grid_convolve
from .green import FOUR_PI


def normals(V, T) -> np.ndarray:
    """Unit normals n_j = (b - a) x (c - a) / |...| of the triangles."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def triangle_dlp(r, a, b, c) -> float:
    """int_T n . (r - r') / |r - r'|^3 dS' in closed form (n the triangle's
    unit normal): sign(h) sum_i [atan(P0 l+ / (R0^2 + |h| R+)) -
    atan(P0 l- / (R0^2 + |h| R-))], the h-derivative of the arctangent part
    of the 1/R edge sum.  0 for points in the plane (principal value)."""
    r = np.asarray(r, dtype=np.float64)
    verts = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    area2 = np.linalg.norm(n)
    n = n / area2
    size = math.sqrt(area2)
    h = float(np.dot(r - verts[0], n))
    ah = abs(h)
    if ah <= 1e-14 * size:
        return 0.0
    rho = r - h * n
    total = 0.0
    for i in range(3):
        pm = verts[i]
        pp = verts[(i + 1) % 3]
        e = pp - pm
        lhat = e / np.linalg.norm(e)
        uhat = np.cross(lhat, n)             # outward in-plane edge normal
        lp = float(np.dot(pp - rho, lhat))
        lm = float(np.dot(pm - rho, lhat))
        P0 = float(np.dot(pm - rho, uhat))   # > 0 when rho is on the inner side
        R0sq = P0 * P0 + h * h
        Rp = float(np.linalg.norm(r - pp))
        Rm = float(np.linalg.norm(r - pm))
        if abs(P0) > 1e-14 * size:
            total += math.atan(P0 * lp / (R0sq + ah * Rp)) - math.atan(P0 * lm / (R0sq + ah * Rm))
    return math.copysign(total, h)


def triangle_dlp_points(r, a, b, c) -> np.ndarray:
    """``triangle_dlp`` for many observation points r[M, 3] (array form of the
    same closed form)."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    verts = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    area2 = np.linalg.norm(n)
    n = n / area2
    size = math.sqrt(area2)
    h = (r - verts[0][None, :]) @ n
    ah = np.abs(h)
    rho = r - h[:, None] * n[None, :]
    total = np.zeros(r.shape[0])
    for i in range(3):
        pm = verts[i]
        pp = verts[(i + 1) % 3]
        lhat = (pp - pm) / np.linalg.norm(pp - pm)
        uhat = np.cross(lhat, n)
        lp = (pp[None, :] - rho) @ lhat
        lm = (pm[None, :] - rho) @ lhat
        P0 = (pm[None, :] - rho) @ uhat
        R0sq = P0 * P0 + h * h
        Rp = np.linalg.norm(r - pp[None, :], axis=1)
        Rm = np.linalg.norm(r - pm[None, :], axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            att = np.arctan(P0 * lp / (R0sq + ah * Rp)) - np.arctan(P0 * lm / (R0sq + ah * Rm))
        total += np.where(np.abs(P0) > 1e-14 * size, att, 0.0)
    return np.where(ah > 1e-14 * size, np.copysign(total, h), 0.0)


def triangle_dlp_quadrature(r, a, b, c, order: int = 60) -> float:
    """The same integral by Gauss-Legendre quadrature on the Duffy map of
    each sub-triangle (rho, p_i, p_i+1), rho the foot of r (for h != 0 the
    integrand is smooth; the map keeps the peak at the foot resolved)."""
    r = np.asarray(r, dtype=np.float64)
    A, B, C = (np.asarray(v, float) for v in (a, b, c))
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    h = float(np.dot(r - A, n))
    rho = r - h * n
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    U, Vv = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    total = 0.0
    vs = [A, B, C]
    full2 = float(np.linalg.norm(np.cross(B - A, C - A)))
    for i in range(3):
        p1, p2 = vs[i], vs[(i + 1) % 3]
        signed2 = float(np.dot(np.cross(p1 - rho, p2 - rho), n))
        if abs(signed2) < 1e-13 * full2:
            continue
        pts = rho[None, None, :] + U[..., None] * (p1 - rho)[None, None, :] \
            + (U * Vv)[..., None] * (p2 - p1)[None, None, :]
        R = np.linalg.norm(pts - r[None, None, :], axis=-1)
        total += signed2 * np.sum(W * U * h / R ** 3)
    return total


def static_near(V, T, rows, cols) -> np.ndarray:
    """K_s,NR[i, j] = sum_p (A_i/3) (1/4 pi) int_{T_j} n_j.(r_ip - r')/R^3 dS'."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty(rows.size)
    for j in np.unique(cols):                       # all pairs of one source triangle
        sel = np.nonzero(cols == j)[0]
        a, b, c = V[T[j, 0]], V[T[j, 1]], V[T[j, 2]]
        vals = triangle_dlp_points(qp[rows[sel]].reshape(-1, 3), a, b, c).reshape(-1, 3)
        out[sel] = (vals * w[rows[sel]]).sum(axis=1) / FOUR_PI
    return out


def grad_kernel(k: float, h: float, static: bool = False):
    """The channels' grid kernel as a function of the integer offset array
    d = u - v (shape [..., 3]): returns [..., 3], component a =
    h d_a (1 + jkR) e^{-jkR} / (4 pi R^3) (static: h d_a / (4 pi R^3)),
    R = h |d|, and 0 at d = 0."""
    def kern(d):
        d = np.asarray(d, dtype=np.float64)
        D = np.linalg.norm(d, axis=-1)
        out = np.zeros(d.shape, dtype=np.complex128)
        nz = D > 0
        R = h * D[nz]
        if static:
            f = h / (FOUR_PI * R ** 3)
        else:
            f = h * (1.0 + 1j * k * R) * np.exp(-1j * k * R) / (FOUR_PI * R ** 3)
        out[nz] = d[nz] * f[:, None]
        return out
    return kern


def precorrection(Pm: sp.csr_matrix, rows, cols, dims, h: float, nrm, kern) -> np.ndarray:
    """sum_u sum_v P[u, i] (H_grad(u - v) . n_j) P[v, j] on the given pairs,
    for a channel kernel kern(d) -> [..., 3] (grad_kernel)."""
    Pc = Pm.tocsc()
    Nx, Ny, _ = dims
    out = np.empty(len(rows), dtype=np.complex128)

    def column(j):
        sl = slice(Pc.indptr[j], Pc.indptr[j + 1])
        u = Pc.indices[sl]
        xyz = np.stack([u % Nx, (u // Nx) % Ny, u // (Nx * Ny)], axis=1).astype(np.float64)
        return xyz, Pc.data[sl]

    for t, (i, j) in enumerate(zip(rows, cols)):
        xi, wi = column(int(i))
        xj, wj = column(int(j))
        Kd = kern(xi[:, None, :] - xj[None, :, :])          # [ni, nj, 3]
        out[t] = wi @ (Kd @ nrm[int(j)]) @ wj
    return out


def circulant_grad_kernels(k: float, dims, h: float) -> np.ndarray:
    """First columns of the circulant embeddings of the three channels'
    kernels, shape (3, 2Nz, 2Ny, 2Nx) (index i on an axis of length M = 2N
    stands for offset i (i < N) or i - M (i > N); index N holds 0)."""
    axes = []
    for N in dims:
        M = 2 * N
        i = np.arange(M)
        d = np.where(i < N, i, i - M).astype(np.float64)
        axes.append((d, i != N))
    (dx, vx), (dy, vy), (dz, vz) = axes
    Dz, Dy, Dx = np.meshgrid(dz, dy, dx, indexing="ij")
    valid = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    d = np.stack([Dx, Dy, Dz], axis=-1)
    K = grad_kernel(k, h)(d)
    K[~valid] = 0.0
    return np.moveaxis(K, -1, 0)


class DlpOracle:
    """AIMx double-layer operator on the mesh, grid, stencils and near list of
    an AimOracle."""

    def __init__(self, aim: AimOracle):
        self.o = aim
        self.n = normals(aim.V, aim.T)
        self._C = None
        self._spec = {}

    def correction_values(self, rows, cols) -> np.ndarray:
        """C_K = K_s,NR - K_s,P on the given pairs (real)."""
        o = self.o
        pre = precorrection(o.P, rows, cols, o.dims, o.h, self.n, grad_kernel(0.0, o.h, True))
        return static_near(o.V, o.T, rows, cols) - pre.real

    @property
    def C(self) -> sp.csr_matrix:
        if self._C is None:
            rows, cols = self.o.near_list()
            self._C = sp.csr_matrix((self.correction_values(rows, cols), (rows, cols)),
                                    shape=(self.o.N, self.o.N))
        return self._C

    def spectra(self, k: float) -> np.ndarray:
        key = float(k)
        if key not in self._spec:
            self._spec[key] = scipy.fft.fftn(circulant_grad_kernels(key, self.o.dims, self.o.h),
                                             axes=(-3, -2, -1), workers=FFT_WORKERS)
        return self._spec[key]

    def far(self, x, k: float) -> np.ndarray:
        """W sum_a H_grad,a(k) P diag(n_a) x."""
        o = self.o
        x = np.asarray(x, dtype=np.complex128)
        S = self.spectra(k)
        phi = 0.0
        for a in range(3):
            phi = phi + grid_convolve(o.project(x * self.n[:, a]), S[a], o.dims)
        return o.interpolate(phi)

    def matvec_rows(self, x, k: float, rows) -> np.ndarray:
        """Selected entries of K x: the far part over the whole grid, the
        correction only on the requested rows."""
        o = self.o
        rows = np.unique(np.asarray(rows, dtype=np.int64))
        rr, cc = o.near_list()
        sel = np.isin(rr, rows)
        vals = self.correction_values(rr[sel], cc[sel])
        Cs = sp.csr_matrix((vals, (rr[sel], cc[sel])), shape=(o.N, o.N))
        x = np.asarray(x, dtype=np.complex128)
        return self.far(x, k)[rows] + (Cs @ x)[rows]

    def matvec(self, x, k: float) -> np.ndarray:
        """y = C_K x + W H_grad(k) P^(K) x (eq. KAIMx)."""
        x = np.asarray(x, dtype=np.complex128)
        y = self.far(x, k)
        if x.ndim == 1:
            return y + self.C @ x
        return y + (self.C @ x.T).T


def dense_rows(V, T, k: float, rows) -> np.ndarray:
    """Rows of the dense double-layer matrix by direct integration: the
    static part by the closed form (principal value on the diagonal), the
    smooth remainder n_j.(r - r')[(1 + jkR) e^{-jkR} - 1]/(4 pi R^3) by the
    3 x 3 point rule (its limit at R = 0 is 0 for in-plane pairs)."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    nrm = normals(V, T)
    N = T.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros((rows.size, N), dtype=np.complex128)
    ro = qp[rows].reshape(-1, 3)                                   # [3 m, 3]
    wo = w[rows]                                                   # [m, 3]
    for j in range(N):
        a, b, c = V[T[j, 0]], V[T[j, 1]], V[T[j, 2]]
        st = (triangle_dlp_points(ro, a, b, c).reshape(-1, 3) * wo).sum(axis=1) / FOUR_PI
        d = qp[rows][:, :, None, :] - qp[j][None, None, :, :]     # [m, 3, 3, 3]
        R = np.linalg.norm(d, axis=-1)
        nd = d @ nrm[j]
        with np.errstate(divide="ignore", invalid="ignore"):
            dyn = np.where(R > 0, nd * ((1.0 + 1j * k * R) * np.exp(-1j * k * R) - 1.0)
                           / (FOUR_PI * np.where(R > 0, R, 1.0) ** 3), 0.0)
        out[:, j] = st + np.sum(wo[:, :, None] * w[j][None, None, :] * dyn, axis=(1, 2))
    return out
