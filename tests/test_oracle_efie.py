"""Pins of the RWG EFIE oracle (Sec. II-A, eq. EFIEdis; Sec. II-B, eq. LAIMx)
against what the mathematics fixes.

* The closed-form vector integral int_T r'/R dS' against quadrature, on and
  off the plane.
* RWG identities: a closed mesh has 3N/2 functions; each function's charge
  integrates to zero; its normal component across its edge is 1 from both
  sides (the current is continuous).
* The precorrection summed over the channels equals the dense grid product
  sum_c P_c^T H_s P_c (and the charge channel alone likewise).
* The dense direct-integration matrix is symmetric (the EFIE's reciprocity).
* The accelerated operator approaches the dense matrix (a few percent at
  h = lambda/10), and more closely on a finer grid with the near region held
  fixed.
"""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx, efie, green, mesh


def test_vector_integral_matches_quadrature():
    a = np.array([0.0, 0.0, 0.0])
    b = np.array([1.0, 0.1, 0.0])
    c = np.array([0.3, 0.9, 0.0])
    rng = np.random.default_rng(3)
    pts = [np.array([rng.uniform(-0.5, 1.5), rng.uniform(-0.5, 1.5), rng.uniform(-1, 1)])
           for _ in range(12)]
    pts += [np.array([0.4, 0.3, 0.0]), np.array([1.2, 1.1, 0.0]), np.array([0.5, 0.05, 0.0])]
    for r in pts:
        ref = efie.triangle_rvec_r_quadrature(r, a, b, c, order=80)
        got = efie.triangle_rvec_r(r, a, b, c)
        assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref)), r


def test_rwg_identities():
    w = I.sphere_tiny(level=2)
    rwg = efie.Rwg(w.vertices, w.triangles)
    N = w.triangles.shape[0]
    assert rwg.n == 3 * N // 2 and np.all(rwg.tri_rwg >= 0)
    V, T = rwg.V, rwg.T
    for n in (0, 17, rwg.n - 1):
        tp, tm = rwg.tp[n], rwg.tm[n]
        ep = int(np.nonzero(rwg.tri_rwg[tp] == n)[0][0])
        em = int(np.nonzero(rwg.tri_rwg[tm] == n)[0][0])
        # zero total charge
        assert rwg.divergence(tp, ep) * rwg.area[tp] + rwg.divergence(tm, em) * rwg.area[tm] \
            == pytest.approx(0.0, abs=1e-14)
        # unit normal component across the edge from both sides: in each
        # triangle's own plane, out of T+ and into T-
        p, q = V[rwg.edges[n, 0]], V[rwg.edges[n, 1]]
        mid = 0.5 * (p + q)
        for t, e, into in ((tp, ep, False), (tm, em, True)):
            m = np.cross(q - p, mesh.unit_normals(V, T)[t])
            m /= np.linalg.norm(m)
            toward_free = np.dot(m, V[T[t, e]] - mid) > 0
            if toward_free != into:
                m = -m
            assert np.dot(rwg.on_triangle(t, e, mid), m) == pytest.approx(1.0, rel=1e-12)


def test_precorrection_equals_dense_grid_product():
    w = I.sphere_tiny(level=1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 10.0)
    e = efie.EfieOracle(o)
    Nx, Ny, Nz = o.dims
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) * o.h
    R = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)
    with np.errstate(divide="ignore"):
        Hs = np.where(R > 0, 1.0 / (4 * math.pi * np.where(R > 0, R, 1.0)), 0.0)
    P = [p.toarray() for p in e.P]
    dense_a = sum(P[c].T @ Hs @ P[c] for c in range(3))
    dense_q = P[3].T @ Hs @ P[3]
    got_a = sum(aimx.precorrection(e.P[c], e.rows, e.cols, o.dims, o.h) for c in range(3))
    got_q = aimx.precorrection(e.P[3], e.rows, e.cols, o.dims, o.h)
    assert e.rows.size == e.n * e.n
    assert np.max(np.abs(got_a - dense_a[e.rows, e.cols])) <= 1e-12 * np.max(np.abs(dense_a))
    assert np.max(np.abs(got_q - dense_q[e.rows, e.cols])) <= 1e-12 * np.max(np.abs(dense_q))


def test_dense_matrix_is_symmetric():
    w = I.sphere_tiny(level=1)
    rwg = efie.Rwg(w.vertices, w.triangles)
    rows = np.arange(0, rwg.n, 5)
    Z = efie.dense_rows(rwg, 2 * math.pi, rows)
    sub = Z[:, rows]
    assert np.max(np.abs(sub - sub.T)) <= 1e-13 * np.max(np.abs(sub))


def test_accelerated_operator_against_dense_reference():
    k = 2 * math.pi
    errs = []
    for dims, hh, tau in (((16, 16, 16), 0.1, 0.3), ((32, 32, 32), 0.05, 0.3)):
        w = I.sphere_tiny(level=2, dims=dims, h=hh, k=k)
        o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, tau)
        e = efie.EfieOracle(o)
        x = I.complex_gaussian(e.n, 23)
        rows = np.arange(0, e.n, 37)
        ref = efie.dense_rows(e.rwg, k, rows, e._cache) @ x
        errs.append(np.linalg.norm(e.matvec_rows(x, k, rows) - ref) / np.linalg.norm(ref))
    print(f"EFIE against the dense matrix: h = 0.1: {errs[0]:.2e}, h = 0.05: {errs[1]:.2e}")
    assert errs[0] <= 0.05
    assert errs[1] < 0.5 * errs[0]


def _diagonals(e, k):
    """Diagonal entries of L^A and L^phi (Z = L^A - L^phi / k^2): AIMx
    (C + the grid product with H(k), self term -jk/(4 pi)) and direct
    integration (static closed form + G_d by the 3 x 3 point rule)."""
    o, rwg = e.o, e.rwg
    Nx, Ny, _ = o.dims
    m_all = np.arange(e.n)
    sa, sphi = efie.static_near(rwg, m_all, m_all, e._cache)
    ca, cq = e.correction_values(m_all, m_all)
    vals = rwg.point_values()
    qp = mesh.quad_points(rwg.V, rwg.T)
    tris = {}
    for t in range(rwg.T.shape[0]):
        for ed in range(3):
            if rwg.tri_rwg[t, ed] >= 0:
                tris.setdefault(int(rwg.tri_rwg[t, ed]), []).append((t, ed))
    Pc = [p.tocsc() for p in e.P]
    out = {"aimx": np.zeros((2, e.n), complex), "direct": np.zeros((2, e.n), complex)}
    for m in range(e.n):
        for c in range(4):                       # grid part of channel c
            sl = slice(Pc[c].indptr[m], Pc[c].indptr[m + 1])
            u, w = Pc[c].indices[sl], Pc[c].data[sl]
            xyz = np.stack([u % Nx, (u // Nx) % Ny, u // (Nx * Ny)], 1).astype(float)
            R = o.h * np.linalg.norm(xyz[:, None] - xyz[None], axis=-1)
            with np.errstate(divide="ignore", invalid="ignore"):
                H = np.where(R > 0, np.exp(-1j * k * R) / (4 * math.pi * np.where(R > 0, R, 1)),
                             -1j * k / (4 * math.pi))
            out["aimx"][0 if c < 3 else 1, m] += w @ H @ w
        dyn = np.zeros(2, complex)
        for tm, em in tris[m]:
            for tn, en in tris[m]:
                R = np.linalg.norm(qp[tm][:, None] - qp[tn][None], axis=-1)
                gd = green.green_dynamic(k, R)
                a, b = vals[tm, :, em, :], vals[tn, :, en, :]
                dyn[0] += np.sum((a[:, :3] @ b[:, :3].T) * gd)
                dyn[1] += np.sum(np.outer(a[:, 3], b[:, 3]) * gd)
        out["direct"][:, m] = [sa[m] + dyn[0], sphi[m] + dyn[1]]
    out["aimx"][0] += ca
    out["aimx"][1] += cq
    return out


def test_diagonal_error_falls_with_frequency():
    """Sec. IV-B's overlap error Delta L = max over the diagonal of
    |L_AIMx - L_direct| / |L_direct|, for L^A, L^phi and the EFIE matrix
    L^A - L^phi/k^2, on a 1 m sphere with a second-order stencil: below 1% at
    edges of about lambda/10, and falling with frequency (the paper's Sec.
    IV-B experiment on its own mesh and grid sizes)."""
    V, T = I.icosphere(2, 0.5)
    edge = float(np.mean(np.linalg.norm(V[T[:, 0]] - V[T[:, 1]], axis=1)))
    res = []
    for frac in (0.1, 0.03):                     # mean edge / wavelength
        k = 2 * math.pi * frac / edge
        o = aimx.AimOracle(V, T, 2, (32, 32, 32), 0.0, 0.3)
        e = efie.EfieOracle(o)
        d = _diagonals(e, k)
        dA = np.max(np.abs(d["aimx"][0] - d["direct"][0]) / np.abs(d["direct"][0]))
        dP = np.max(np.abs(d["aimx"][1] - d["direct"][1]) / np.abs(d["direct"][1]))
        za, zd = d["aimx"][0] - d["aimx"][1] / k ** 2, d["direct"][0] - d["direct"][1] / k ** 2
        dZ = np.max(np.abs(za - zd) / np.abs(zd))
        res.append((dA, dP, dZ))
        print(f"edge = {frac} lambda: Delta L^A {dA:.2e}, L^phi {dP:.2e}, EFIE {dZ:.2e}")
    assert max(res[0]) < 1e-2
    assert all(res[1][i] < res[0][i] for i in range(3))
