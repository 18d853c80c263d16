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
from oracle import aimx, efie, mesh


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
