"""The AIMx operator, step by step, in float64/complex128 (oracle).

Scalar single-layer operator with one piecewise-constant basis function per
triangle and Galerkin testing -- the scalar-potential structure of the
discretised EFIE (Sec. II-A, eq. EFIEdis) -- accelerated as in eq. LAIMx:

    A(k) x  ~=  A_s,NR x  -  A_s,P x  +  W H(k) P x

* P  projects quadrature-point sources onto grid stencils (Sec. II-B,
     eq. aimLFR); for every quadrature point the weights are the tensor
     Lagrange polynomials of its (n+1)^3 stencil, which is the moment-matching
     projection (Sec. IV, equivalence to polynomial interpolation).
* H  is the three-level Toeplitz matrix of G(k, r_m - r_n) over grid points
     (eq. Hmn) with the self term replaced by -jk/(4 pi) (eq. Hmm); its
     product runs as a zero-padded circulant FFT convolution (Sec. II-B).
* W  = P^T (Galerkin testing with the same scalar basis).
* A_s,NR is the near-region matrix of the static kernel G_s (eq. hgfs) by
  direct integration (analytic inner integral, 3-point outer rule, then
  symmetrised); A_s,P = W H_s,NR P is its precorrection (eq. aimLPs) with
  H_s self term 0 (eq. Hsmm).  C = A_s,NR - A_s,P is real and independent of
  frequency (Sec. III-A).

Readings where the paper is silent (stencil placement, grid placement,
padding, near criterion) are fixed in the docstrings below.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.sparse as sp
from scipy.spatial import cKDTree

from . import mesh as _mesh
from .green import FOUR_PI, green_full
from .potential import triangle_inv_r_points, triangle_potential

FFT_WORKERS = -1   # all host cores


class GridError(ValueError):
    """A stencil leaves the grid."""


# --------------------------------------------------------------------------
# grid and stencils
# --------------------------------------------------------------------------

def grid_spacing(V, dims, h: float) -> float:
    """Isotropic spacing: ``h`` if positive, else the smallest spacing that
    fits the vertex bounding box into ``dims`` with two spare nodes per side,
    h = max_a extent_a / (N_a - 5)."""
    if h > 0:
        return float(h)
    ext = V.max(axis=0) - V.min(axis=0)
    return float(max(ext[a] / (dims[a] - 5) for a in range(3)))


def grid_origin(V, dims, h: float) -> np.ndarray:
    """Grid centred on the vertex bounding box:
    origin_a = (min_a + max_a)/2 - h (N_a - 1)/2."""
    lo = V.min(axis=0)
    hi = V.max(axis=0)
    dims = np.asarray(dims, dtype=np.float64)
    return 0.5 * (lo + hi) - h * (dims - 1.0) / 2.0


def stencil_start(points, origin, h: float, order: int, dims):
    """First node s and local coordinate u = t - s of each point per axis.

    t = (x - origin)/h; s = floor(t - (n-1)/2), so the n+1 nodes s..s+n
    straddle t symmetrically (n+1 points per direction, Sec. IV-A).  Raises
    GridError if any stencil is not inside 0..N-1.
    """
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    t = (pts - origin[None, :]) / h
    s = np.floor(t - (order - 1) / 2.0).astype(np.int64)
    dims = np.asarray(dims, dtype=np.int64)
    if (s < 0).any() or (s + order > dims[None, :] - 1).any():
        raise GridError("a projection stencil leaves the grid")
    return s, t - s


def lagrange_weights(u, order: int):
    """l_a(u) = prod_{b != a} (u - b) / (a - b) for a = 0..n, shape [..., n+1]."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty(u.shape + (order + 1,))
    for a in range(order + 1):
        w = np.ones(u.shape)
        for b in range(order + 1):
            if b != a:
                w = w * (u - b) / (a - b)
        out[..., a] = w
    return out


def node_index(ix, iy, iz, dims):
    """Flat grid index, x fastest: ix + Nx (iy + Ny iz)."""
    return ix + dims[0] * (iy + dims[1] * iz)


def projection_matrix(V, T, order: int, dims, h: float, origin) -> sp.csr_matrix:
    """P[u, j] = sum_q (A_j/3) Lambda_u(r_jq)  (sparse, Ng x N).

    Lambda_u(r) = l_a(u_x) l_b(u_y) l_c(u_z) for node u = s + (a, b, c).
    """
    N = T.shape[0]
    qp = _mesh.quad_points(V, T).reshape(-1, 3)
    w = _mesh.quad_weights(V, T).reshape(-1)
    s, u = stencil_start(qp, origin, h, order, dims)
    L = lagrange_weights(u, order)          # [M, 3, n+1]
    rows, cols, vals = [], [], []
    tri = np.repeat(np.arange(N), 3)
    for a in range(order + 1):
        for b in range(order + 1):
            for c in range(order + 1):
                rows.append(node_index(s[:, 0] + a, s[:, 1] + b, s[:, 2] + c, dims))
                cols.append(tri)
                vals.append(w * L[:, 0, a] * L[:, 1, b] * L[:, 2, c])
    Ng = int(np.prod(dims))
    Pm = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(Ng, N))
    return Pm.tocsr()


# --------------------------------------------------------------------------
# Toeplitz kernel and FFT convolution
# --------------------------------------------------------------------------

def circulant_kernel(k: float, dims, h: float) -> np.ndarray:
    """First column of the circulant embedding of H(k), shape (2Nz, 2Ny, 2Nx).

    Index i on an axis of padded length M = 2N stands for the grid offset
    d = i (i < N) or i - M (i > N); entry G(k, h|d|) for d != 0 (eq. Hmn)
    and -jk/(4 pi) for d = 0 (eq. Hmm).  Index i = N is never reached by a
    linear convolution of two length-N sequences and holds 0.
    """
    axes = []
    for N in dims:
        M = 2 * N
        i = np.arange(M)
        d = np.where(i < N, i, i - M).astype(np.float64)
        valid = i != N
        axes.append((d, valid))
    (dx, vx), (dy, vy), (dz, vz) = axes
    D = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
    valid = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    R = h * D
    c = np.zeros(D.shape, dtype=np.complex128)
    nz = valid & (D > 0)
    c[nz] = green_full(k, R[nz])
    c[0, 0, 0] = -1j * k / FOUR_PI
    return c


def kernel_spectrum(k: float, dims, h: float) -> np.ndarray:
    """H_hat = FFT3(circulant kernel) (numpy sign convention)."""
    return scipy.fft.fftn(circulant_kernel(k, dims, h), workers=FFT_WORKERS)


def grid_convolve(q, Hhat, dims):
    """phi = H q over the unpadded grid by zero-padded circulant FFT.

    ``q`` has shape (Nz, Ny, Nx) (or a leading batch axis); returns phi of
    the same shape.
    """
    Nx, Ny, Nz = dims
    q = np.asarray(q)
    batch = q.shape[:-3]
    g = np.zeros(batch + (2 * Nz, 2 * Ny, 2 * Nx), dtype=np.complex128)
    g[..., :Nz, :Ny, :Nx] = q
    G = scipy.fft.fftn(g, axes=(-3, -2, -1), workers=FFT_WORKERS)
    phi = scipy.fft.ifftn(Hhat * G, axes=(-3, -2, -1), workers=FFT_WORKERS)
    return phi[..., :Nz, :Ny, :Nx]


def grid_convolve_bruteforce(q, k: float, dims, h: float):
    """phi[m] = sum_n H(r_m - r_n) q[n] by direct summation (tiny grids only),
    H(0) = -jk/(4 pi)."""
    Nx, Ny, Nz = dims
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64) * h
    R = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)
    H = np.empty(R.shape, dtype=np.complex128)
    off = R > 0
    H[off] = green_full(k, R[off])
    H[~off] = -1j * k / FOUR_PI
    return (H @ np.asarray(q).reshape(-1)).reshape(Nz, Ny, Nx)


# --------------------------------------------------------------------------
# near region
# --------------------------------------------------------------------------

def near_pairs(cent, tau: float):
    """All ordered pairs (i, j), self pairs included, whose centroids are
    closer than tau (strict).  Returns (rows, cols) sorted by row then col."""
    tree = cKDTree(cent)
    pairs = tree.query_pairs(r=tau, output_type="ndarray")
    if pairs.size:
        d = np.linalg.norm(cent[pairs[:, 0]] - cent[pairs[:, 1]], axis=1)
        pairs = pairs[d < tau]
    N = cent.shape[0]
    rows = np.concatenate([np.arange(N), pairs[:, 0], pairs[:, 1]]).astype(np.int64)
    cols = np.concatenate([np.arange(N), pairs[:, 1], pairs[:, 0]]).astype(np.int64)
    order = np.lexsort((cols, rows))
    return rows[order], cols[order]


def static_near_entry(V, T, i: int, j: int, qp=None, w=None) -> float:
    """M_ij = sum_p (A_i/3) Phi_j(r_ip): 3-point outer rule on triangle i,
    closed-form inner potential of triangle j.  ``qp``/``w`` may carry the
    precomputed quadrature points [N,3,3] and weights [N,3]."""
    if qp is None:
        qp = _mesh.quad_points(V, T)
        w = _mesh.quad_weights(V, T)
    a, b, c = V[T[j, 0]], V[T[j, 1]], V[T[j, 2]]
    return float(sum(w[i, p] * triangle_potential(qp[i, p], a, b, c) for p in range(3)))


def static_near(V, T, rows, cols) -> np.ndarray:
    """Entries of A_s,NR = (M + M^T)/2 on the given pairs (grouped by the
    source triangle so that each closed-form call covers many points)."""
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    # every (i, j) and (j, i) that is needed
    need_i = np.concatenate([rows, cols])
    need_j = np.concatenate([cols, rows])
    order = np.lexsort((need_i, need_j))
    need_i, need_j = need_i[order], need_j[order]
    M = {}
    bounds = np.flatnonzero(np.diff(need_j)) + 1
    for grp in np.split(np.arange(need_j.size), bounds):
        if grp.size == 0:
            continue
        j = int(need_j[grp[0]])
        ii = np.unique(need_i[grp])
        a, b, c = V[T[j, 0]], V[T[j, 1]], V[T[j, 2]]
        phi = triangle_inv_r_points(qp[ii].reshape(-1, 3), a, b, c).reshape(-1, 3) / FOUR_PI
        vals = np.sum(w[ii] * phi, axis=1)
        for t, i in enumerate(ii):
            M[(int(i), j)] = float(vals[t])
    return np.array([0.5 * (M[(int(i), int(j))] + M[(int(j), int(i))])
                     for i, j in zip(rows, cols)])


def precorrection(Pm: sp.csr_matrix, rows, cols, dims, h: float) -> np.ndarray:
    """Entries of A_s,P = W H_s,NR P on the given pairs (eq. aimLPs), pairs
    sorted by row:
    sum_u sum_v P[u,i] H_s(r_u - r_v) P[v,j] with H_s(R) = 1/(4 pi R) and
    H_s(0) = 0 (eq. Hsmm)."""
    Pc = Pm.tocsc()
    Nx, Ny, _ = dims
    vals = np.empty(rows.size)
    cache = {}

    def col(j):
        if j not in cache:
            sl = slice(Pc.indptr[j], Pc.indptr[j + 1])
            u = Pc.indices[sl]
            w = Pc.data[sl]
            xyz = np.stack([u % Nx, (u // Nx) % Ny, u // (Nx * Ny)], axis=1).astype(np.float64)
            cache[j] = (xyz, w)
        return cache[j]

    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    bounds = np.flatnonzero(np.diff(rows)) + 1
    for grp in np.split(np.arange(rows.size), bounds):
        if grp.size == 0:
            continue
        xi, wi = col(int(rows[grp[0]]))
        blocks = [col(int(j)) for j in cols[grp]]
        xj = np.concatenate([b[0] for b in blocks])
        wj = np.concatenate([b[1] for b in blocks])
        seg = np.repeat(np.arange(grp.size), [b[1].size for b in blocks])
        R = h * np.linalg.norm(xi[:, None, :] - xj[None, :, :], axis=-1)
        Hs = np.where(R > 0, 1.0 / (FOUR_PI * np.where(R > 0, R, 1.0)), 0.0)
        contrib = (wi @ Hs) * wj
        vals[grp] = np.bincount(seg, weights=contrib, minlength=grp.size)
    return vals


# --------------------------------------------------------------------------
# the operator
# --------------------------------------------------------------------------

class AimOracle:
    """The AIMx operator of eq. LAIMx for one mesh and grid.

    Parameters follow the library's setup call: vertices, triangles, stencil
    order n, unpadded grid dims (Nx, Ny, Nz), spacing h (<= 0: derived) and
    the near-region threshold (absolute length; centroid distance < tau).
    """

    def __init__(self, V, T, order: int, dims, h: float, tau: float):
        self.V = np.asarray(V, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.order = int(order)
        self.dims = tuple(int(d) for d in dims)
        self.h = grid_spacing(self.V, self.dims, h)
        self.tau = float(tau)
        self.origin = grid_origin(self.V, self.dims, self.h)
        self.N = self.T.shape[0]
        self.P = projection_matrix(self.V, self.T, self.order, self.dims, self.h, self.origin)
        self.cent = _mesh.centroids(self.V, self.T)
        self._C = None
        self._spectra = {}

    # -- pieces ------------------------------------------------------------
    def stencils(self):
        qp = _mesh.quad_points(self.V, self.T).reshape(-1, 3)
        return stencil_start(qp, self.origin, self.h, self.order, self.dims)

    def spectrum(self, k: float) -> np.ndarray:
        key = float(k)
        if key not in self._spectra:
            self._spectra[key] = kernel_spectrum(key, self.dims, self.h)
        return self._spectra[key]

    def project(self, x) -> np.ndarray:
        """q = P x on the unpadded grid, shape (Nz, Ny, Nx) (or batched)."""
        x = np.asarray(x)
        Nx, Ny, Nz = self.dims
        if x.ndim == 1:
            return (self.P @ x).reshape(Nz, Ny, Nx)
        return (self.P @ x.T).T.reshape(x.shape[0], Nz, Ny, Nx)

    def interpolate(self, phi) -> np.ndarray:
        """y = P^T phi."""
        phi = np.asarray(phi)
        if phi.ndim == 3:
            return self.P.T @ phi.reshape(-1)
        return (self.P.T @ phi.reshape(phi.shape[0], -1).T).T

    def far(self, x, k: float) -> np.ndarray:
        """W H(k) P x."""
        return self.interpolate(grid_convolve(self.project(x), self.spectrum(k), self.dims))

    def near_list(self):
        return near_pairs(self.cent, self.tau)

    def correction_rows(self, rows_wanted):
        """Rows of C = A_s,NR - A_s,P for the requested basis functions, as
        (rows, cols, vals)."""
        rows_wanted = np.unique(np.asarray(rows_wanted, dtype=np.int64))
        tree = cKDTree(self.cent)
        rr, cc = [], []
        for i in rows_wanted:
            nb = np.array(sorted(tree.query_ball_point(self.cent[i], self.tau)), dtype=np.int64)
            d = np.linalg.norm(self.cent[nb] - self.cent[i], axis=1)
            nb = nb[(d < self.tau) | (nb == i)]
            rr.append(np.full(nb.size, i))
            cc.append(nb)
        rows = np.concatenate(rr)
        cols = np.concatenate(cc)
        vals = static_near(self.V, self.T, rows, cols) - \
            precorrection(self.P, rows, cols, self.dims, self.h)
        return rows, cols, vals

    @property
    def C(self) -> sp.csr_matrix:
        """The full correction matrix (small problems only)."""
        if self._C is None:
            rows, cols = self.near_list()
            vals = static_near(self.V, self.T, rows, cols) - \
                precorrection(self.P, rows, cols, self.dims, self.h)
            self._C = sp.csr_matrix((vals, (rows, cols)), shape=(self.N, self.N))
        return self._C

    def static_near_matrix(self) -> sp.csr_matrix:
        """A_s,NR alone (used for the static preconditioners of Sec. III-A)."""
        rows, cols = self.near_list()
        vals = static_near(self.V, self.T, rows, cols)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.N, self.N))

    def matvec(self, x, k: float) -> np.ndarray:
        """y = A_s,NR x - A_s,P x + W H(k) P x (eq. LAIMx)."""
        x = np.asarray(x, dtype=np.complex128)
        y = self.far(x, k)
        if x.ndim == 1:
            return y + self.C @ x
        return y + (self.C @ x.T).T

    def matvec_rows(self, x, k: float, rows):
        """Selected entries of A x: the far part over the whole grid, the
        correction only on the requested rows (large problems)."""
        rows = np.asarray(rows, dtype=np.int64)
        yfar = self.far(x, k)
        r, c, v = self.correction_rows(rows)
        Cs = sp.csr_matrix((v, (r, c)), shape=(self.N, self.N))
        return yfar[rows] + (Cs @ np.asarray(x, dtype=np.complex128))[rows]
