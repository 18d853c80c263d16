"""Pins of the conventional-AIM oracle (Sec. II-B) against what the
mathematics fixes.

* The precorrection W H_NR(k) P equals the explicit product P^T H P of a
  brute-force dense H on a tiny grid.
* Small-k structure of C(k) - C (conventional minus AIMx correction), from
  the Taylor series of G_d (eq. hgfdtaylor) and moment matching of the
  stencils (Sec. IV): the k-linear term -jk/(4 pi) cancels exactly because
  the Lagrange weights of a stencil sum to one and the 3-point weights of a
  triangle sum to its area (both sides give -jk/(4 pi) A_i A_j; it would not
  cancel with any other grid self term); the k^3 R^2 term cancels too,
  because a stencil of order n >= 2 reproduces quadratics; so the real part
  of C(k) - C is O(k^2) (from -k^2 R/(8 pi), eq. linterm) and the imaginary
  part O(k^5).
* The near entries are those of the dense reference; complex symmetry.
"""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx, mesh
from oracle.conventional import (ConventionalAim, dynamic_near, full_grid_kernel,
                                 precorrection_with)
from oracle.dense import dense_rows
from oracle.green import FOUR_PI, green_full


def test_precorrection_with_static_kernel_is_the_aimx_precorrection():
    w = I.sphere_tiny()
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    rows, cols = o.near_list()
    ref = aimx.precorrection(o.P, rows, cols, o.dims, o.h)

    def static(R):
        return np.where(R > 0, 1.0 / (FOUR_PI * np.where(R > 0, R, 1.0)), 0.0)
    got = precorrection_with(o.P, rows, cols, o.dims, o.h, static)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_full_precorrection_equals_dense_grid_product():
    """With a threshold above the diameter every pair of the 80-triangle
    sphere is near, so A_P(k) must equal P^T H P with H the full dense grid
    matrix."""
    w = I.sphere_tiny()
    k = 5.3
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 10.0)
    rows, cols = o.near_list()
    assert rows.size == o.N * o.N
    Nx, Ny, Nz = o.dims
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) * o.h
    D = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)
    H = np.full(D.shape, -1j * k / FOUR_PI)
    off = D > 0
    H[off] = green_full(k, D[off])
    Pd = o.P.toarray()
    dense = Pd.T @ H @ Pd
    got = precorrection_with(o.P, rows, cols, o.dims, o.h, full_grid_kernel(k))
    ref = dense[rows, cols]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def sphere_rows():
    w = I.sphere_small()
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    rows, cols = o.near_list()
    sel = rows < 60
    return w, o, rows[sel], cols[sel]


def test_small_k_structure_of_the_difference_to_aimx(sphere_rows):
    w, o, rows, cols = sphere_rows
    conv = ConventionalAim(o)
    c_aimx = aimx.static_near(o.V, o.T, rows, cols) - \
        aimx.precorrection(o.P, rows, cols, o.dims, o.h)
    diffs = {}
    for k in (0.05, 0.1, 0.2):
        diffs[k] = conv.correction_values(rows, cols, k) - c_aimx
    re = {k: np.linalg.norm(d.real) for k, d in diffs.items()}
    im = {k: np.linalg.norm(d.imag) for k, d in diffs.items()}
    # real part ~ k^2, imaginary part ~ k^5 (the k and k^3 terms cancel)
    assert re[0.1] / re[0.05] == pytest.approx(4.0, rel=2e-3)
    assert re[0.2] / re[0.1] == pytest.approx(4.0, rel=5e-3)
    assert im[0.2] / im[0.1] == pytest.approx(32.0, rel=2e-2)
    # the k^2 coefficient is -(1/(8 pi)) (sum w w R - P^T R P) on each pair
    lin = precorrection_with(o.P, rows, cols, o.dims, o.h, lambda R: R.astype(np.complex128))
    q = mesh.quad_points(o.V, o.T)
    wq = mesh.quad_weights(o.V, o.T)
    R = np.linalg.norm(q[rows][:, :, None, :] - q[cols][:, None, :, :], axis=-1)
    direct = np.sum(wq[rows][:, :, None] * wq[cols][:, None, :] * R, axis=(1, 2))
    coef = -(direct - lin.real) / (8.0 * math.pi)
    k = 0.05
    assert np.linalg.norm(diffs[k].real - k * k * coef) <= 2e-3 * np.linalg.norm(k * k * coef)


def test_near_entries_are_those_of_the_dense_reference(sphere_rows):
    w, o, rows, cols = sphere_rows
    k = float(w.k[0])
    ns = o.static_near_matrix()
    D = dense_rows(o.V, o.T, k, np.arange(3), ns)
    sel = rows < 3
    anr = aimx.static_near(o.V, o.T, rows[sel], cols[sel]) + \
        dynamic_near(o.V, o.T, rows[sel], cols[sel], k)
    assert np.max(np.abs(anr - D[rows[sel], cols[sel]])) <= 1e-14 * np.max(np.abs(anr))


def test_correction_is_complex_symmetric():
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, 0.25)
    C = ConventionalAim(o).correction(6.0).toarray()
    assert np.max(np.abs(C - C.T)) <= 1e-13 * np.max(np.abs(C))


def test_conventional_is_at_least_as_accurate_as_aimx_against_the_dense_reference():
    """The far operator is shared, and the conventional AIM integrates the
    whole near region directly while AIMx takes its dynamic part from the
    grid (Sec. III-A), so against the dense direct-quadrature matrix the
    conventional operator is no less accurate; the gap grows with k h (the
    accuracy discussion of Sec. III-A and Sec. IV-B)."""
    from oracle.dense import dense_matvec
    w = I.sphere_small()
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    conv = ConventionalAim(o)
    ns = o.static_near_matrix()
    x = I.complex_gaussian(o.N, 11)
    rows = np.arange(0, o.N, 7)
    errs = {}
    for k in (2 * math.pi, 10.0):
        yd = dense_matvec(o.V, o.T, k, x, ns, rows)
        ea = np.linalg.norm(o.matvec(x, k)[rows] - yd) / np.linalg.norm(yd)
        ec = np.linalg.norm(conv.matvec(x, k)[rows] - yd) / np.linalg.norm(yd)
        errs[k] = (ea, ec)
        assert ec <= ea
        assert ea <= 0.05
    assert errs[10.0][0] - errs[10.0][1] > errs[2 * math.pi][0] - errs[2 * math.pi][1]
