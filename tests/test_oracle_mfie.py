"""Pins of the RWG double-layer (MFIE) oracle (Sec. III-B, eqs. opK, ghgf,
KAIMx) against what the mathematics fixes.

* The closed-form static gradient integral int_T (r - r')/R^3 against
  quadrature off the triangle; its normal part against the solid angle of
  the scalar double layer; its in-plane part against finite differences of
  the closed-form 1/R potential (so also in the plane of T, where the
  normal part is the principal value 0); its far-field limit.
* On a flat mesh the integrand of K is normal to the plane, so the static
  entries and the dense matrix vanish (to rounding) for every k.
* The grid field sum_v H_grad(u - v) x J(v) by six FFT convolutions equals
  the direct sum on tiny grids; the precorrection equals the dense grid
  product W^T H_grad,s x P.
* The Gram matrix equals high-order quadrature of f_m . f_n.
* The accelerated operator approaches the dense direct-integration matrix,
  more closely on a finer grid with the near region held fixed.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2009_02281_amd import inputs as I
from oracle import aimx, dlp, efie, mesh, mfie
from oracle.potential import triangle_inv_r


def tri():
    return (np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0]), np.array([0.3, 0.9, 0.0]))


def test_closed_form_against_quadrature_and_far_limit():
    a, b, c = tri()
    rng = np.random.default_rng(5)
    for _ in range(15):
        r = np.array([rng.uniform(-0.5, 1.5), rng.uniform(-0.5, 1.5), 0.0])
        r[2] = rng.choice([-1, 1]) * rng.uniform(0.1, 1.0)
        ref = mfie.triangle_grad_inv_r_quadrature(r, a, b, c)
        got = mfie.triangle_grad_inv_r(r, a, b, c)
        assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref)), r
    for r in (np.array([1.6, 1.2, 0.0]), np.array([-0.4, 0.5, 0.0])):   # in plane, outside
        ref = mfie.triangle_grad_inv_r_quadrature(r, a, b, c, order=120)
        assert np.max(np.abs(mfie.triangle_grad_inv_r(r, a, b, c) - ref)) <= 1e-9 * np.max(
            np.abs(ref))
    cen = (a + b + c) / 3
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    d = np.array([40.0, -30.0, 50.0])
    far = mfie.triangle_grad_inv_r(cen + d, a, b, c)
    assert np.allclose(far, area * d / np.linalg.norm(d) ** 3, rtol=1e-3)


def test_normal_part_is_the_solid_angle_and_in_plane_part_the_gradient():
    a, b, c = tri()
    n = np.array([0.0, 0.0, 1.0])
    pts = [np.array([0.4, 0.3, 0.0]), np.array([0.4, 0.3, 0.2]), np.array([1.3, -0.2, -0.4]),
           np.array([0.35, 0.5, 0.0]), np.array([1.2, 1.1, 0.0])]
    eps = 1e-5
    for r in pts:
        g = mfie.triangle_grad_inv_r(r, a, b, c)
        assert g @ n == pytest.approx(dlp.triangle_dlp(r, a, b, c), rel=1e-12, abs=1e-14)
        # int (r - r')/R^3 = -grad_r int 1/R; in-plane components by central differences
        for ax in (0, 1):
            e = np.zeros(3)
            e[ax] = eps
            fd = -(triangle_inv_r(r + e, a, b, c) - triangle_inv_r(r - e, a, b, c)) / (2 * eps)
            assert g[ax] == pytest.approx(fd, rel=1e-6, abs=1e-8), (r, ax)
    inside = pts[0]
    for h in (1e-9, -1e-9):
        g = mfie.triangle_grad_inv_r(inside + [0, 0, h], a, b, c)
        assert g[2] == pytest.approx(math.copysign(2 * math.pi, h), rel=1e-6)
        assert np.allclose(g[:2], mfie.triangle_grad_inv_r(inside, a, b, c)[:2], rtol=1e-6)
    assert mfie.triangle_grad_inv_r(inside, a, b, c)[2] == 0.0     # principal value


def test_static_entries_against_the_definition():
    """K_s,NR on pairs of functions whose triangles do not touch, against the
    definition f_m . (n x int grad G_s x f_n dS') with the same 3-point outer
    rule and Gauss quadrature for the inner integral."""
    w = I.sphere_tiny(level=1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 10.0)
    m = mfie.MfieOracle(efie.EfieOracle(o))
    rwg = m.rwg
    V, T = rwg.V, rwg.T
    qp = mesh.quad_points(V, T)
    wq = mesh.quad_weights(V, T)
    nrm = mesh.unit_normals(V, T)
    x, wts = np.polynomial.legendre.leggauss(30)
    x, wts = 0.5 * (x + 1), 0.5 * wts
    U, Vv = np.meshgrid(x, x, indexing="ij")
    W2 = np.outer(wts, wts)
    tris = m._tris
    count = 0
    for mm in range(0, rwg.n, 7):
        for nn in range(3, rwg.n, 11):
            vm = {int(v) for t, _ in tris[mm] for v in T[t]}
            vn = {int(v) for t, _ in tris[nn] for v in T[t]}
            if vm & vn:
                continue
            ref = 0.0
            for tm, em in tris[mm]:
                for q in range(3):
                    r = qp[tm, q]
                    field = np.zeros(3)
                    for tn, en in tris[nn]:
                        A, B, C = (V[T[tn, i]] for i in range(3))
                        pts = A + U[..., None] * (B - A) + (U * Vv)[..., None] * (C - B)
                        jac = 2 * rwg.area[tn] * U
                        d = r - pts
                        R = np.linalg.norm(d, axis=-1)
                        gs = -d / (4 * math.pi * R[..., None] ** 3)
                        fn = rwg.on_triangle(tn, en, pts)
                        field += np.einsum("ij,ijk->k", W2 * jac, np.cross(gs, fn))
                    ref += wq[tm, q] * np.dot(rwg.on_triangle(tm, em, r),
                                              np.cross(nrm[tm], field))
            got = m.static_entry(mm, nn)
            assert got == pytest.approx(ref, rel=1e-9, abs=1e-12 * abs(ref) + 1e-15), (mm, nn)
            count += 1
    assert count >= 10


def flat_plate():
    n = 5
    xs = np.linspace(-0.4, 0.4, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    a, b, c, d = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel(), idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    T = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    return V, T


def test_flat_mesh_has_no_double_layer():
    V, T = flat_plate()
    o = aimx.AimOracle(V, T, 2, (16, 16, 8), 0.1, 10.0)     # every pair near
    m = mfie.MfieOracle(efie.EfieOracle(o))
    rows = np.arange(0, m.n, 6)
    K = mfie.dense_rows(m.rwg, 2 * math.pi, rows, m)
    G = m.gram(np.repeat(rows, m.n), np.tile(np.arange(m.n), rows.size))
    assert np.max(np.abs(K)) <= 1e-14 * np.max(np.abs(G))


def test_grid_field_equals_direct_sum():
    w = I.sphere_tiny(level=1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 10.0)
    m = mfie.MfieOracle(efie.EfieOracle(o))
    k = 5.3
    x = I.complex_gaussian(m.n, 61)
    Nx, Ny, Nz = o.dims
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    H = -dlp.grad_kernel(k, o.h)(pts[:, None, :] - pts[None, :, :])     # grad G samples
    J = np.stack([m.J[c] @ x for c in range(3)], axis=1)                # [Ng, 3]
    Vf = np.cross(H, J[None, :, :]).sum(axis=1)
    ref = sum(m.Wt[a].T @ Vf[:, a] for a in range(3))
    got = m.far(x, k)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_precorrection_equals_dense_grid_product():
    w = I.sphere_tiny(level=1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 10.0)
    m = mfie.MfieOracle(efie.EfieOracle(o))
    Nx, Ny, Nz = o.dims
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    Hs = -dlp.grad_kernel(0.0, o.h, True)(pts[:, None, :] - pts[None, :, :]).real
    Jd = np.stack([p.toarray() for p in m.J], axis=-1)                 # [Ng, n, 3]
    Wd = np.stack([p.toarray() for p in m.Wt], axis=-1)
    sel = np.arange(0, m.rows.size, 41)
    rows, cols = m.rows[sel], m.cols[sel]
    got = m.precorrection(rows, cols)
    ref = np.array([np.sum(Wd[:, i, :] * np.cross(Hs, Jd[None, :, j, :]).sum(axis=1))
                    for i, j in zip(rows, cols)])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gram_against_quadrature():
    w = I.sphere_tiny(level=1)
    rwg = efie.Rwg(w.vertices, w.triangles)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 10.0)
    m = mfie.MfieOracle(efie.EfieOracle(o))
    x, wts = np.polynomial.legendre.leggauss(8)
    x, wts = 0.5 * (x + 1), 0.5 * wts
    pairs = [(0, 0), (3, 3), (5, 17)]
    for t, e1 in ((0, 0), (7, 1)):
        pairs.append((int(rwg.tri_rwg[t, e1]), int(rwg.tri_rwg[t, (e1 + 1) % 3])))
    got = m.gram([p[0] for p in pairs], [p[1] for p in pairs])
    for (mm, nn), g in zip(pairs, got):
        ref = 0.0
        for t in range(rwg.T.shape[0]):
            es = {int(rwg.tri_rwg[t, e]): e for e in range(3)}
            if mm in es and nn in es:
                A, B, C = (rwg.V[rwg.T[t, i]] for i in range(3))
                for u, wu in zip(x, wts):
                    for v, wv in zip(x, wts):
                        r = A + u * (B - A) + u * v * (C - B)
                        jac = 2 * rwg.area[t] * u
                        ref += wu * wv * jac * np.dot(rwg.on_triangle(t, es[mm], r),
                                                      rwg.on_triangle(t, es[nn], r))
        assert g == pytest.approx(ref, rel=1e-12), (mm, nn)


def test_accelerated_operator_against_dense_reference():
    k = 2 * math.pi
    errs = []
    for dims, hh in (((16, 16, 16), 0.1), ((32, 32, 32), 0.05)):
        w = I.sphere_tiny(level=2, dims=dims, h=hh, k=k)
        o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 0.3)
        m = mfie.MfieOracle(efie.EfieOracle(o))
        x = I.complex_gaussian(m.n, 62)
        rows = np.arange(0, m.n, 37)
        ref = mfie.dense_rows(m.rwg, k, rows, m) @ x
        errs.append(np.linalg.norm(m.matvec_rows(x, k, rows) - ref) / np.linalg.norm(ref))
    print(f"K against the dense matrix: h = 0.1: {errs[0]:.2e}, h = 0.05: {errs[1]:.2e}")
    assert errs[0] <= 0.05
    assert errs[1] < 0.5 * errs[0]


def test_plane_wave_vectors_at_zero_frequency():
    """At k = 0 the tested field is pol . int f_m, which is exact under the
    3-point rule: int_T (r - p) = A (c - p), so int f_m = (l/2)[(c+ - p+) +
    (p- - c-)]."""
    w = I.sphere_tiny(level=1)
    rwg = efie.Rwg(w.vertices, w.triangles)
    pol = np.array([0.3, -0.7, 0.2])
    b = efie.plane_wave_tested(rwg, 0.0, [0, 0, 1], pol)
    cen = mesh.centroids(rwg.V, rwg.T)
    for m in range(rwg.n):
        tp, tm = rwg.tp[m], rwg.tm[m]
        ep = int(np.nonzero(rwg.tri_rwg[tp] == m)[0][0])
        em = int(np.nonzero(rwg.tri_rwg[tm] == m)[0][0])
        pp, pm = rwg.V[rwg.T[tp, ep]], rwg.V[rwg.T[tm, em]]
        ref = 0.5 * rwg.length[m] * ((cen[tp] - pp) + (pm - cen[tm])) @ pol
        assert b[m] == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_magnetic_and_electric_field_equations_agree_on_a_sphere():
    """Physics fixes the signs: for a plane wave on a closed sphere, the
    tested MFIE (G/2 - K) J = <f, n x H_inc> (K the principal value, residue
    -G/2) and the tested EFIE j k Z J = <f, E_inc> (eta0 = 1) give the same
    current, up to the MFIE's discretisation error (5% here); the other
    sign choices of K and the residue miss by far more."""
    k = 2 * math.pi * 0.8
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1, k=k)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    e = efie.EfieOracle(o)
    m = mfie.MfieOracle(e)
    n = e.n
    Z = np.zeros((n, n), complex)
    K = np.zeros((n, n), complex)
    CA, CP = e.corrections()
    CK = sp.csr_matrix((m.correction_values(m.rows, m.cols), (m.rows, m.cols)), shape=(n, n))
    G = sp.csr_matrix((m.gram(m.rows, m.cols), (m.rows, m.cols)), shape=(n, n)).toarray()
    for j in range(n):
        x = np.zeros(n, complex)
        x[j] = 1.0
        Z[:, j] = e.far(x, k) + CA @ x - CP @ x / k ** 2
        K[:, j] = m.far(x, k) + CK @ x
    d, pol = [0, 0, 1], [1, 0, 0]
    bE = efie.plane_wave_tested(e.rwg, k, d, pol, "E")
    bH = efie.plane_wave_tested(e.rwg, k, d, pol, "H")
    JE = np.linalg.solve(Z, bE / (1j * k))
    errs = {}
    for sgn in (1, -1):
        for beta in (-0.5, 0.5):
            JM = np.linalg.solve(-sgn * (K + beta * G), bH)
            errs[(sgn, beta)] = np.linalg.norm(JM - JE) / np.linalg.norm(JE)
    print("MFIE against EFIE:", {k2: round(v, 3) for k2, v in errs.items()})
    assert errs[(1, -0.5)] < 0.08
    assert min(v for k2, v in errs.items() if k2 != (1, -0.5)) > 0.5
    # the combined field Z + (j/k)(K - G/2) with (bE + bH)/(jk) gives the same current
    JC = np.linalg.solve(Z + 1j / k * (K - 0.5 * G), (bE + bH) / (1j * k))
    assert np.linalg.norm(JC - JE) / np.linalg.norm(JE) < 0.05
