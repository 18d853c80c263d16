"""Pins of the oracle's AIMx operator: projection moments, FFT convolution vs
brute force, precorrection vs a dense double loop, symmetry, accuracy vs
the dense direct-quadrature matrix, the scalar sphere series, and the
solver vs a direct factorisation."""
import math
import os

import numpy as np
import pytest
from scipy.special import eval_legendre

from paper_2009_02281_amd import inputs as I
from oracle import aimx, dense, excitation, mesh, mie, solver
from oracle.green import FOUR_PI, green_full

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mpmath_values.txt")


def test_projection_matches_moments(sphere_oracle):
    """sum_u P[u,j] m(r_u) = sum_q w_q m(r_q) for every monomial of degree
    <= n per axis (moment matching of the quadrature sources, Sec. II-B)."""
    w, o = sphere_oracle
    Nx, Ny, Nz = o.dims
    u = np.arange(Nx * Ny * Nz)
    xyz = np.stack([u % Nx, (u // Nx) % Ny, u // (Nx * Ny)], axis=1) * o.h + o.origin
    qp = mesh.quad_points(o.V, o.T)
    wq = mesh.quad_weights(o.V, o.T)
    c = o.cent
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                # monomials centred per basis keep the numbers O(1)
                m_grid = None
                lhs = np.empty(o.N)
                P = o.P.tocsc()
                for j in range(0, o.N, 97):
                    sl = slice(P.indptr[j], P.indptr[j + 1])
                    d = xyz[P.indices[sl]] - c[j]
                    lhs[j] = np.sum(P.data[sl] * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** cc)
                    dq = qp[j] - c[j]
                    rhs = np.sum(wq[j] * dq[:, 0] ** a * dq[:, 1] ** b * dq[:, 2] ** cc)
                    assert lhs[j] == pytest.approx(rhs, abs=1e-14 * wq[j].sum())
    # a moment of degree n+1 along one axis is not matched in general
    j = 5
    sl = slice(P.indptr[j], P.indptr[j + 1])
    d = xyz[P.indices[sl]] - c[j]
    dq = qp[j] - c[j]
    assert abs(np.sum(P.data[sl] * d[:, 0] ** 3) - np.sum(wq[j] * dq[:, 0] ** 3)) > 1e-9


@pytest.mark.parametrize("dims", [(3, 4, 5), (4, 4, 4), (5, 2, 3)])
def test_fft_convolution_equals_bruteforce(dims):
    rng = np.random.default_rng(sum(dims))
    k, h = 2 * math.pi, 0.13
    q = rng.standard_normal(dims[::-1]) + 1j * rng.standard_normal(dims[::-1])
    fast = aimx.grid_convolve(q, aimx.kernel_spectrum(k, dims, h), dims)
    slow = aimx.grid_convolve_bruteforce(q, k, dims, h)
    assert np.max(np.abs(fast - slow)) <= 1e-13 * np.max(np.abs(slow))


def test_padding_entry_is_irrelevant():
    """The circulant entry at index N never enters the product."""
    dims, k, h = (4, 3, 5), 2.0, 0.2
    rng = np.random.default_rng(4)
    q = rng.standard_normal(dims[::-1]) + 0j
    c = aimx.circulant_kernel(k, dims, h)
    c2 = c.copy()
    c2[dims[2], :, :] = 7.0
    c2[:, dims[1], :] = -3.0 + 1j
    c2[:, :, dims[0]] = 11.0
    import scipy.fft as F
    a = aimx.grid_convolve(q, F.fftn(c), dims)
    b = aimx.grid_convolve(q, F.fftn(c2), dims)
    assert np.max(np.abs(a - b)) < 1e-13


def test_self_term_is_modified_kernel():
    """H(0) = -jk/(4 pi) (eq. Hmm): a unit grid source sees it at its own
    node and G(k, h) at a neighbour."""
    dims, k, h = (5, 5, 5), 3.0, 0.1
    q = np.zeros(dims[::-1], dtype=complex)
    q[2, 2, 2] = 1.0
    phi = aimx.grid_convolve(q, aimx.kernel_spectrum(k, dims, h), dims)
    assert phi[2, 2, 2] == pytest.approx(-1j * k / FOUR_PI, abs=1e-14)
    assert phi[2, 2, 3] == pytest.approx(complex(green_full(k, h)), rel=1e-12)


def test_precorrection_equals_dense_double_loop(sphere_oracle):
    w, o = sphere_oracle
    rows, cols = o.near_list()
    pick = np.random.default_rng(5).choice(rows.size, 25, replace=False)
    Pd = o.P.tocsc()
    Nx, Ny, _ = o.dims
    vals = aimx.precorrection(o.P, rows, cols, o.dims, o.h)
    for t in pick:
        i, j = rows[t], cols[t]
        ref = 0.0
        for a in range(Pd.indptr[i], Pd.indptr[i + 1]):
            for b in range(Pd.indptr[j], Pd.indptr[j + 1]):
                u, v = Pd.indices[a], Pd.indices[b]
                du = np.array([u % Nx - v % Nx, (u // Nx) % Ny - (v // Nx) % Ny,
                               u // (Nx * Ny) - v // (Nx * Ny)], dtype=float)
                R = o.h * np.linalg.norm(du)
                if R > 0:
                    ref += Pd.data[a] * Pd.data[b] / (FOUR_PI * R)
        assert vals[t] == pytest.approx(ref, rel=1e-12)


def test_precorrection_far_pair_approximates_point_rule(sphere_oracle):
    """For well-separated triangles W H_s P ~ the 3x3 point rule of G_s
    (interpolation error only)."""
    w, o = sphere_oracle
    i, j = 0, int(np.argmax(np.linalg.norm(o.cent - o.cent[0], axis=1)))
    pc = aimx.precorrection(o.P, np.array([i]), np.array([j]), o.dims, o.h)[0]
    qp = mesh.quad_points(o.V, o.T)
    wq = mesh.quad_weights(o.V, o.T)
    R = np.linalg.norm(qp[i][:, None] - qp[j][None], axis=-1)
    ref = np.sum(wq[i][:, None] * wq[j][None] / (FOUR_PI * R))
    assert pc == pytest.approx(ref, rel=1e-3)


def test_correction_is_real_symmetric_and_static(sphere_oracle):
    w, o = sphere_oracle
    C = o.C
    assert C.dtype == np.float64
    assert abs(C - C.T).max() <= 1e-15 * abs(C).max()
    # nnz per row of the near list (centroid distance < 2h) is ~52 here
    assert 40 < C.nnz / o.N < 70


def test_operator_complex_symmetric(sphere_oracle):
    w, o = sphere_oracle
    k = 2 * math.pi
    x = I.complex_gaussian(o.N, 11)
    y = I.complex_gaussian(o.N, 12)
    lhs = x @ o.matvec(y, k)
    rhs = y @ o.matvec(x, k)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_row_sampled_matvec_equals_full(sphere_oracle):
    w, o = sphere_oracle
    k = 2 * math.pi
    x = I.complex_gaussian(o.N, 1001)
    rows = np.array([0, 17, 640, 1279])
    full = o.matvec(x, k)
    samp = o.matvec_rows(x, k, rows)
    assert np.max(np.abs(full[rows] - samp)) <= 1e-14 * np.max(np.abs(full))


def test_close_to_dense_reference_and_converges_with_grid():
    """AIMx vs the dense direct-quadrature operator: about 1% at h = 0.1
    (10 points per wavelength; Sec. IV-B reports < 1% at 0.1 lambda edges),
    and smaller on a finer grid (grid refinement controls the error)."""
    V, T = I.icosphere(2, 0.5)
    k = 2 * math.pi
    x = I.complex_gaussian(T.shape[0], 21)
    errs = []
    for dims, h in [((16, 16, 16), 0.1), ((28, 28, 28), 0.05)]:
        o = aimx.AimOracle(V, T, 2, dims, h, 0.2)
        ns = o.static_near_matrix()
        yd = dense.dense_matvec(V, T, k, x, ns)
        ya = o.matvec(x, k)
        errs.append(np.linalg.norm(ya - yd) / np.linalg.norm(yd))
    assert errs[0] < 2e-2
    assert errs[1] < 0.5 * errs[0]


def test_dense_reference_symmetric_and_diagonal():
    V, T = I.icosphere(1, 0.5)
    o = aimx.AimOracle(V, T, 2, (8, 8, 8), 0.2, 0.4)
    ns = o.static_near_matrix()
    D = dense.dense_rows(V, T, 2 * math.pi, np.arange(T.shape[0]), ns)
    assert np.max(np.abs(D - D.T)) <= 1e-14 * np.max(np.abs(D))
    # far entries are the 3x3 point rule of the full kernel
    qp, wq = mesh.quad_points(V, T), mesh.quad_weights(V, T)
    i, j = 0, int(np.argmax(np.linalg.norm(o.cent - o.cent[0], axis=1)))
    R = np.linalg.norm(qp[i][:, None] - qp[j][None], axis=-1)
    ref = np.sum(wq[i][:, None] * wq[j][None] * green_full(2 * math.pi, R))
    assert D[i, j] == pytest.approx(ref, rel=1e-13)


# -- scalar sphere series

def test_series_kernel_matches_closed_form():
    k = 2 * math.pi
    rng = np.random.default_rng(7)
    for _ in range(5):
        # the series converges like (r</r>)^l; keep the radii apart
        r1, r2 = rng.uniform(0.3, 0.5), rng.uniform(0.8, 1.0)
        cg = rng.uniform(-1, 1)
        R = math.sqrt(r1 * r1 + r2 * r2 - 2 * r1 * r2 * cg)
        got = mie.green_series(k, r1, r2, cg, lmax=120)
        assert got == pytest.approx(complex(green_full(k, R)), rel=1e-11)


def test_series_eigenvalues_match_arbitrary_precision():
    with open(GOLDEN) as f:
        rows = [list(map(float, ln.split()[1:])) for ln in f if ln.startswith("lam ")]
    for l, k, a, re, im in rows:
        assert mie.eigenvalue(int(l), k, a) == pytest.approx(complex(re, im), rel=1e-12)


def test_operator_eigenvalues_on_sphere(sphere_oracle):
    """A applied to P_l(cos theta) on the mesh, divided by the test areas,
    reproduces lam_l P_l for l >= 1 within discretisation error."""
    w, o = sphere_oracle
    k = 2 * math.pi
    A = mesh.areas(o.V, o.T)
    ct = o.cent[:, 2] / np.linalg.norm(o.cent, axis=1)
    for l in (1, 2, 3):
        x = eval_legendre(l, ct).astype(complex)
        lam = mie.eigenvalue(l, k, 0.5)
        err = np.linalg.norm(o.matvec(x, k) / A - lam * x) / np.linalg.norm(lam * x)
        assert err < 3e-2


@pytest.mark.slow
def test_operator_eigenvalues_improve_with_refinement():
    k = 2 * math.pi
    errs = []
    for lev, dims, h in [(3, (16, 16, 16), 0.1), (4, (24, 24, 24), 0.06)]:
        V, T = I.icosphere(lev, 0.5)
        o = aimx.AimOracle(V, T, 2, dims, h, 2 * h)
        A = mesh.areas(V, T)
        c = mesh.centroids(V, T)
        ct = c[:, 2] / np.linalg.norm(c, axis=1)
        x = eval_legendre(2, ct).astype(complex)
        lam = mie.eigenvalue(2, k, 0.5)
        errs.append(np.linalg.norm(o.matvec(x, k) / A - lam * x) / np.linalg.norm(lam * x))
    assert errs[1] < 0.5 * errs[0]


def test_plane_wave_rhs_integral():
    """sum_i b_i ~ integral of exp(-jkz) over the sphere = 4 pi a^2 j0(ka)."""
    V, T = I.icosphere(4, 0.5)
    for k in (0.9 * 2 * math.pi, 2 * math.pi):
        b = excitation.plane_wave(V, T, k)
        ka = k * 0.5
        exact = 4 * math.pi * 0.25 * math.sin(ka) / ka
        assert abs(b.sum() - exact) < 1e-2 * 4 * math.pi * 0.25


def test_gmres_matches_direct_solve_and_mie(sphere_oracle):
    """GMRES on the AIMx system: the solution matches a direct solve of the
    assembled operator, and its exterior field matches the sphere series."""
    w, o = sphere_oracle
    k = 2 * math.pi
    b = excitation.plane_wave(o.V, o.T, k)
    x, info = solver.fgmres(lambda v: o.matvec(v, k), b, tol=1e-8, restart=30, max_iter=3000)
    assert info.converged and info.rel_resid <= 1e-8
    Afull = np.empty((o.N, o.N), dtype=complex)
    eye = np.eye(o.N)
    for j in range(0, o.N, 128):
        Afull[:, j:j + 128] = o.matvec(eye[j:j + 128].astype(complex), k).T
    xd = np.linalg.solve(Afull, b)
    # rigorous: ||x - x_direct|| <= ||b - A x|| / sigma_min(A)
    smin = np.linalg.svd(Afull, compute_uv=False)[-1]
    resid = np.linalg.norm(b - Afull @ x)
    assert resid <= 1.01e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - xd) <= 1.01 * resid / smin + 1e-12 * np.linalg.norm(xd)
    # exterior field at r = 2a
    th = np.linspace(0.1, math.pi - 0.1, 9)
    pts = np.stack([np.sin(th), 0 * th, np.cos(th)], 1) * 1.0
    qp, wq = mesh.quad_points(o.V, o.T), mesh.quad_weights(o.V, o.T)
    R = np.linalg.norm(pts[:, None, None, :] - qp[None], axis=-1)
    u = np.sum(green_full(k, R) * wq[None] * x[None, :, None], axis=(1, 2))
    ue = mie.exterior_field_plane_wave(k, 0.5, 1.0, np.cos(th))
    assert np.linalg.norm(u - ue) / np.linalg.norm(ue) < 3e-2


def test_diagonal_preconditioner_from_static_matrix(sphere_oracle):
    """The static diagonal (Sec. III-A) is a valid right preconditioner:
    the preconditioned solve reaches the same solution."""
    w, o = sphere_oracle
    k = 2 * math.pi * 0.9
    b = excitation.plane_wave(o.V, o.T, k)
    d = o.static_near_matrix().diagonal()
    x1, i1 = solver.fgmres(lambda v: o.matvec(v, k), b, tol=1e-10, restart=30, max_iter=3000)
    x2, i2 = solver.fgmres(lambda v: o.matvec(v, k), b, tol=1e-10, restart=30, max_iter=3000,
                           M=lambda v: v / d)
    assert i1.converged and i2.converged
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-7


def test_gmres_small_dense_textbook():
    rng = np.random.default_rng(0)
    n = 50
    A = np.eye(n) * 3 + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 0j
    for m in (5, 50):
        x, info = solver.fgmres(lambda v: A @ v, b, tol=1e-12, restart=m, max_iter=400)
        assert info.converged
        assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)


def test_cluster_block_is_the_dense_reference_restricted_to_the_cluster():
    """The near-block preconditioner's block (full kernel: static near
    entries plus the dynamic part) equals the dense reference matrix on the
    cluster's rows and columns, and is complex symmetric."""
    from oracle.dense import cluster_block, dense_rows
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 0.25)
    ns = o.static_near_matrix()
    members = np.array([3, 7, 11, 40, 41, 100, 200])
    k = 6.0
    B = cluster_block(o.V, o.T, k, members, ns)
    D = dense_rows(o.V, o.T, k, members, ns)[:, members]
    assert np.max(np.abs(B - D)) <= 1e-14 * np.max(np.abs(D))
    assert np.max(np.abs(B - B.T)) <= 1e-14 * np.max(np.abs(B))
