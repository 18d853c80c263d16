"""The vector EFIE operator with RWG basis functions under AIMx (oracle; test
infrastructure only, used by tests/ and nothing in the library).

Sec. II-A (eq. EFIEdis) discretises the EFIE with RWG basis functions f_n
(Rao, Wilton and Glisson, 1982) and Galerkin testing; with the gradient moved
to the testing function the operator is L^A + k^{-2} L^phi, i.e.

    Z_mn = int int f_m(r) . f_n(r') G dS' dS - (1/k^2) int int (div f_m)(div' f_n) G dS' dS

(the factor -j omega mu is left out).  Sec. II-B projects the sources of
both parts onto the grid: three Cartesian current channels and one charge
channel, all through the same spectrum H(k) (eqs. aimLFR, LAIMx):

    Z ~= C_A - k^{-2} C_phi + sum_{c=x,y,z} P_c^T H(k) P_c - k^{-2} P_q^T H(k) P_q,

with P_c[u, n] = sum over the points q of T_n+ and T_n- of w_q f_{n,c}(r_q)
Lambda_u(r_q) and P_q the same with div f_n; C_A = A_s,NR - A_s,P and
C_phi likewise, from the static kernel (eq. hgfs) on near pairs and its
precorrection with H_s (self term 0, eq. Hsmm) -- both real and frequency
independent, as for the scalar operator (Sec. III-A).

RWG function n lives on the interior edge shared by triangles T+ and T-
(T+ the one of lower index), with length l and the vertices p+-, opposite
the edge:  f_n = l/(2A+) (r - p+) on T+,  l/(2A-) (p- - r) on T-;
div f_n = +l/A+ on T+, -l/A- on T-.  Edges of one triangle only (open
surfaces) carry no function.

Readings (the paper leaves them to standard practice): the static inner
integrals in closed form, int_T 1/R (oracle.potential) and
int_T r'/R dS' = rho int_T 1/R + sum_i u_i int_{edge i} R dl (u_i the outward
in-plane edge normal, rho the foot of r; the gradient theorem for
grad_s' R = (rho' - rho)/R), the outer integral by the 3-point rule, and the
near block symmetrised, (M + M^T)/2; two RWG functions are near when some
triangle of one is near some triangle of the other (the scalar path's
centroid criterion).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import mesh as _mesh
from .aimx import (AimOracle, grid_convolve, lagrange_weights, near_pairs, node_index,
                   precorrection, stencil_start)
from .green import FOUR_PI, green_dynamic
from .potential import triangle_inv_r


# --------------------------------------------------------------------------
# RWG functions
# --------------------------------------------------------------------------

class Rwg:
    """RWG functions of a triangle mesh.  tri_rwg[t, e] is the function on
    the edge of triangle t opposite its vertex e (-1: a boundary edge), and
    tri_sign[t, e] is +1 when t is that function's T+, -1 for T-."""

    def __init__(self, V, T):
        self.V = np.asarray(V, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        N = self.T.shape[0]
        owners = {}
        for t in range(N):
            for e in range(3):
                a, b = int(self.T[t, (e + 1) % 3]), int(self.T[t, (e + 2) % 3])
                owners.setdefault((min(a, b), max(a, b)), []).append((t, e))
        self.tri_rwg = -np.ones((N, 3), dtype=np.int64)
        self.tri_sign = np.zeros((N, 3))
        edges, tp, tm, lengths = [], [], [], []
        for key in sorted(owners):
            own = owners[key]
            if len(own) == 1:
                continue
            if len(own) != 2:
                raise ValueError("an edge is shared by more than two triangles")
            (t1, e1), (t2, e2) = sorted(own)
            n = len(edges)
            edges.append(key)
            tp.append(t1)
            tm.append(t2)
            lengths.append(np.linalg.norm(self.V[key[1]] - self.V[key[0]]))
            self.tri_rwg[t1, e1], self.tri_sign[t1, e1] = n, 1.0
            self.tri_rwg[t2, e2], self.tri_sign[t2, e2] = n, -1.0
        self.edges = np.array(edges, dtype=np.int64).reshape(-1, 2)
        self.tp = np.array(tp, dtype=np.int64)
        self.tm = np.array(tm, dtype=np.int64)
        self.length = np.array(lengths)
        self.n = len(edges)
        self.area = _mesh.areas(self.V, self.T)

    def on_triangle(self, t: int, e: int, r) -> np.ndarray:
        """f_n(r) (r[..., 3] on triangle t) for the function on edge e of t."""
        n = self.tri_rwg[t, e]
        s = self.tri_sign[t, e]
        free = self.V[self.T[t, e]]
        return s * self.length[n] / (2.0 * self.area[t]) * (np.asarray(r) - free)

    def divergence(self, t: int, e: int) -> float:
        n = self.tri_rwg[t, e]
        return self.tri_sign[t, e] * self.length[n] / self.area[t]

    def point_values(self):
        """Per quadrature point of every triangle and local edge: the
        function's four channel values (f_x, f_y, f_z, div f) times the
        point's weight; shape [N, 3 points, 3 edges, 4]."""
        qp = _mesh.quad_points(self.V, self.T)
        w = _mesh.quad_weights(self.V, self.T)
        N = self.T.shape[0]
        out = np.zeros((N, 3, 3, 4))
        for t in range(N):
            for e in range(3):
                if self.tri_rwg[t, e] < 0:
                    continue
                out[t, :, e, :3] = self.on_triangle(t, e, qp[t]) * w[t][:, None]
                out[t, :, e, 3] = self.divergence(t, e) * w[t]
        return out


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def triangle_rvec_r(r, a, b, c) -> np.ndarray:
    """int_T r' / |r - r'| dS' (vector) in closed form: rho int_T 1/R plus
    sum_i u_i [l R + R0^2 ln(l + R)]/2 between each edge's endpoints."""
    r = np.asarray(r, dtype=np.float64)
    verts = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    n = n / np.linalg.norm(n)
    h = float(np.dot(r - verts[0], n))
    rho = r - h * n
    out = rho * triangle_inv_r(r, *verts)
    for i in range(3):
        p, q = verts[i], verts[(i + 1) % 3]
        L = float(np.linalg.norm(q - p))
        t = (q - p) / L
        m = np.cross(t, n)                      # outward in-plane edge normal
        P0 = float(np.dot(p - rho, m))
        lm = float(np.dot(p - rho, t))
        lp = float(np.dot(q - rho, t))
        R0sq = P0 * P0 + h * h
        Rm = float(np.linalg.norm(p - r))
        Rp = float(np.linalg.norm(q - r))
        if R0sq <= (1e-14 * L) ** 2:
            lg = 0.0                            # r on the edge line: R0^2 ln(...) -> 0
        elif lm >= 0.0:
            lg = math.log((Rp + lp) / (Rm + lm))
        elif lp <= 0.0:
            lg = math.log((Rm - lm) / (Rp - lp))
        else:
            lg = math.log((Rp + lp) * (Rm - lm) / R0sq)
        out = out + m * 0.5 * (lp * Rp - lm * Rm + R0sq * lg)
    return out


def triangle_rvec_r_quadrature(r, a, b, c, order: int = 60) -> np.ndarray:
    """The same integral by Gauss-Legendre quadrature on the Duffy map of the
    sub-triangles (rho, p_i, p_i+1) (the 1/R peak at the foot is resolved)."""
    r = np.asarray(r, dtype=np.float64)
    A, B, C = (np.asarray(v, float) for v in (a, b, c))
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    rho = r - np.dot(r - A, n) * n
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    U, Vv = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    full2 = float(np.linalg.norm(np.cross(B - A, C - A)))
    total = np.zeros(3)
    vs = [A, B, C]
    for i in range(3):
        p1, p2 = vs[i], vs[(i + 1) % 3]
        signed2 = float(np.dot(np.cross(p1 - rho, p2 - rho), n))
        if abs(signed2) < 1e-13 * full2:
            continue
        pts = rho[None, None, :] + U[..., None] * (p1 - rho)[None, None, :] \
            + (U * Vv)[..., None] * (p2 - p1)[None, None, :]
        R = np.linalg.norm(pts - r[None, None, :], axis=-1)
        total += signed2 * np.einsum("ij,ijk->k", W * U / R, pts)
    return total


# --------------------------------------------------------------------------
# the operator
# --------------------------------------------------------------------------

def rwg_near_pairs(rwg: Rwg, tri_rows, tri_cols):
    """RWG pairs (m, n) with some triangle of m near some triangle of n,
    sorted by row then column."""
    A = rwg.tri_rwg[np.asarray(tri_rows)]          # [p, 3]
    B = rwg.tri_rwg[np.asarray(tri_cols)]
    m = np.repeat(A, 3, axis=1).ravel()
    n = np.tile(B, (1, 3)).ravel()
    keep = (m >= 0) & (n >= 0)
    key = np.unique(m[keep] * rwg.n + n[keep])
    return key // rwg.n, key % rwg.n


def _inner(rwg: Rwg, tm: int, tn: int, cache: dict):
    """For the 3 quadrature points of triangle tm: int_{tn} 1/R and
    int_{tn} r'/R (closed forms), cached per triangle pair."""
    key = (tm, tn)
    if key not in cache:
        V, T = rwg.V, rwg.T
        qp = _mesh.quad_points(V, T[[tm]])[0]
        a, b, c = (V[T[tn, i]] for i in range(3))
        s1 = np.array([triangle_inv_r(qp[q], a, b, c) for q in range(3)])
        sv = np.array([triangle_rvec_r(qp[q], a, b, c) for q in range(3)])
        cache[key] = (s1, sv)
    return cache[key]


def static_near(rwg: Rwg, rows, cols, cache=None):
    """(A^A_s, A^phi_s) on the RWG pairs: 3-point outer rule on the testing
    function's triangles, closed-form inner integrals, then symmetrised."""
    V, T = rwg.V, rwg.T
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    cache = {} if cache is None else cache
    tris = {}
    for t in range(T.shape[0]):
        for e in range(3):
            n = rwg.tri_rwg[t, e]
            if n >= 0:
                tris.setdefault(int(n), []).append((t, e))

    def entry(m, n):
        aa = ap = 0.0
        for tm, em in tris[m]:
            fm = rwg.on_triangle(tm, em, qp[tm])            # [3, 3]
            dm = rwg.divergence(tm, em)
            for tn, en in tris[n]:
                s1, sv = _inner(rwg, tm, tn, cache)
                free = V[T[tn, en]]
                coef = rwg.tri_sign[tn, en] * rwg.length[n] / (2.0 * rwg.area[tn])
                inner = coef * (sv - free[None, :] * s1[:, None])   # [3, 3]
                aa += np.sum(w[tm] * np.sum(fm * inner, axis=1)) / FOUR_PI
                ap += np.sum(w[tm] * s1) * dm * rwg.divergence(tn, en) / FOUR_PI
        return aa, ap

    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    memo = {}
    outa = np.empty(rows.size)
    outp = np.empty(rows.size)
    for t, (m, n) in enumerate(zip(rows, cols)):
        for key in ((int(m), int(n)), (int(n), int(m))):
            if key not in memo:
                memo[key] = entry(*key)
        outa[t] = 0.5 * (memo[(int(m), int(n))][0] + memo[(int(n), int(m))][0])
        outp[t] = 0.5 * (memo[(int(m), int(n))][1] + memo[(int(n), int(m))][1])
    return outa, outp


def channel_projections(rwg: Rwg, aim: AimOracle, vals=None):
    """P_c, c = x, y, z, q (sparse Ng x n_rwg): sum over the functions'
    quadrature points of w_q g_c(r_q) Lambda_u(r_q); vals [N, 3, 3, C]
    replaces the channel values (default rwg.point_values())."""
    V, T = rwg.V, rwg.T
    qp = _mesh.quad_points(V, T).reshape(-1, 3)
    s, u = stencil_start(qp, aim.origin, aim.h, aim.order, aim.dims)
    L = lagrange_weights(u, aim.order)                  # [Nq, 3, n+1]
    if vals is None:
        vals = rwg.point_values()                       # [N, 3, 3, 4]
    N = T.shape[0]
    S = aim.order + 1
    out = []
    for c in range(vals.shape[-1]):
        rr, cc, vv = [], [], []
        for e in range(3):
            fn = np.repeat(rwg.tri_rwg[:, e], 3)        # per point
            gv = vals[:, :, e, c].reshape(-1)
            ok = fn >= 0
            for a in range(S):
                for b in range(S):
                    for d in range(S):
                        node = node_index(s[:, 0] + a, s[:, 1] + b, s[:, 2] + d, aim.dims)
                        rr.append(node[ok])
                        cc.append(fn[ok])
                        vv.append((gv * L[:, 0, a] * L[:, 1, b] * L[:, 2, d])[ok])
        Ng = int(np.prod(aim.dims))
        out.append(sp.coo_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))),
                                 shape=(Ng, rwg.n)).tocsr())
    return out


class EfieOracle:
    """The AIMx EFIE on the mesh, grid, stencils and near criterion of an
    AimOracle."""

    def __init__(self, aim: AimOracle):
        self.o = aim
        self.rwg = Rwg(aim.V, aim.T)
        self.n = self.rwg.n
        self.P = channel_projections(self.rwg, aim)
        tr, tc = aim.near_list()
        self.rows, self.cols = rwg_near_pairs(self.rwg, tr, tc)
        self._C = None
        self._cache = {}

    def correction_values(self, rows, cols):
        """(C_A, C_phi) on the given RWG pairs."""
        o = self.o
        sa, sphi = static_near(self.rwg, rows, cols, self._cache)
        pa = sum(precorrection(self.P[c], rows, cols, o.dims, o.h) for c in range(3)).real
        pq = precorrection(self.P[3], rows, cols, o.dims, o.h).real
        return sa - pa, sphi - pq

    def corrections(self):
        """(C_A, C_phi) as sparse matrices on the RWG near list."""
        if self._C is None:
            ca, cq = self.correction_values(self.rows, self.cols)
            shape = (self.n, self.n)
            self._C = (sp.csr_matrix((ca, (self.rows, self.cols)), shape=shape),
                       sp.csr_matrix((cq, (self.rows, self.cols)), shape=shape))
        return self._C

    def far(self, x, k: float) -> np.ndarray:
        o = self.o
        Nx, Ny, Nz = o.dims
        S = o.spectrum(k)
        y = 0.0
        for c in range(4):
            q = (self.P[c] @ x).reshape(Nz, Ny, Nx)
            phi = grid_convolve(q, S, o.dims).reshape(-1)
            yc = self.P[c].T @ phi
            y = y + (yc if c < 3 else -yc / (k * k))
        return y

    def matvec_rows(self, x, k: float, rows) -> np.ndarray:
        """Selected entries of Z x: the far part over the whole grid, the
        correction only on the requested rows."""
        rows = np.unique(np.asarray(rows, dtype=np.int64))
        sel = np.isin(self.rows, rows)
        r, c = self.rows[sel], self.cols[sel]
        ca, cq = self.correction_values(r, c)
        Cs = sp.csr_matrix((ca - cq / (k * k), (r, c)), shape=(self.n, self.n))
        x = np.asarray(x, dtype=np.complex128)
        return self.far(x, k)[rows] + (Cs @ x)[rows]

    def matvec(self, x, k: float) -> np.ndarray:
        """Z x = (C_A - C_phi/k^2) x + sum_c P_c^T H P_c x - P_q^T H P_q x / k^2."""
        x = np.asarray(x, dtype=np.complex128)
        CA, CP = self.corrections()
        return self.far(x, k) + CA @ x - (CP @ x) / (k * k)


def dense_rows(rwg: Rwg, k: float, rows, cache=None) -> np.ndarray:
    """Rows of the dense EFIE matrix by direct integration: the static kernel
    in closed form (then symmetrised), the smooth remainder G_d by the 3 x 3
    point rule (G_d(0) = -jk/(4 pi))."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.arange(rwg.n)
    R, Cc = np.meshgrid(rows, cols, indexing="ij")
    sa, sphi = static_near(rwg, R.ravel(), Cc.ravel(), cache)
    out = (sa - sphi / (k * k)).astype(np.complex128).reshape(rows.size, rwg.n)
    V, T = rwg.V, rwg.T
    qp = _mesh.quad_points(V, T)
    vals = rwg.point_values()                           # weights included
    tris = {}
    for t in range(T.shape[0]):
        for e in range(3):
            if rwg.tri_rwg[t, e] >= 0:
                tris.setdefault(int(rwg.tri_rwg[t, e]), []).append((t, e))
    for a, m in enumerate(rows):
        for n in range(rwg.n):
            acc = 0.0
            for tm, em in tris[int(m)]:
                for tn, en in tris[n]:
                    Rr = np.linalg.norm(qp[tm][:, None, :] - qp[tn][None, :, :], axis=-1)
                    Gd = green_dynamic(k, Rr)
                    gm, gn = vals[tm, :, em, :], vals[tn, :, en, :]
                    ff = gm[:, :3] @ gn[:, :3].T
                    dd = np.outer(gm[:, 3], gn[:, 3])
                    acc += np.sum((ff - dd / (k * k)) * Gd)
            out[a, n] += acc
    return out


def plane_wave_tested(rwg: Rwg, k: float, direction, pol, field: str = "E") -> np.ndarray:
    """The incident plane wave E = pol e^{-jk d.r} (d the unit direction)
    tested with the RWG functions by the 3-point rule: field "E" gives
    <f_m, E>; field "H" gives <f_m, n x (d x E)> = eta0 <f_m, n x H>
    (H = d x E / eta0, n the unit normal of each triangle)."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    p = np.asarray(pol, dtype=np.float64)
    qp = _mesh.quad_points(rwg.V, rwg.T)
    vals = rwg.point_values()
    nrm = _mesh.unit_normals(rwg.V, rwg.T)
    out = np.zeros(rwg.n, dtype=np.complex128)
    for t in range(rwg.T.shape[0]):
        vec = p if field == "E" else np.cross(nrm[t], np.cross(d, p))
        ph = np.exp(-1j * k * (qp[t] @ d))
        for e in range(3):
            m = rwg.tri_rwg[t, e]
            if m >= 0:
                out[m] += np.sum((vals[t, :, e, :3] @ vec) * ph)
    return out
