"""Pins of the linear-term modification (Sec. III-A, eqs. linterm and
Lmatdecomplin): the closed-form integral of R over a triangle against
quadrature at points on and off its plane, the grid term against a dense
product, and the accuracy gain the paper reports (AIMx with the term is
closer to the direct matrix whose self entries integrate the linear term
exactly than AIMx without it)."""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx
from oracle.dense import dense_matvec, self_lin_correction
from oracle.lin import (lin_diagonal, lin_grid_kernel, matvec_with_lin, triangle_r_integral,
                        triangle_r_integral_quadrature)


def test_r_integral_closed_form_matches_quadrature():
    rng = np.random.default_rng(41)
    a, b, c = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0]), np.array([0.3, 0.8, 0.0])
    pts = [np.array([0.4, 0.3, 0.0]),            # inside, on the plane
           np.array([0.6, 0.4, 0.0]),            # inside
           np.array([1.5, -0.2, 0.0]),           # outside, on the plane
           np.array([0.5, 0.05, 0.0]),           # near an edge
           np.array([0.0, 0.0, 0.0])]            # at a vertex
    pts += [rng.uniform(-0.5, 1.5, 3) for _ in range(6)]
    pts += [np.array([0.4, 0.3, 1e-3]), np.array([0.4, 0.3, -0.7])]
    for r in pts:
        ref = triangle_r_integral_quadrature(r, a, b, c)
        got = triangle_r_integral(r, a, b, c)
        assert abs(got - ref) <= 1e-10 * abs(ref), r


def test_r_integral_far_limit_and_centroid_moment():
    """Far away the integral tends to A |r - c| with c the centroid (the
    first moment of the triangle about its centroid vanishes)."""
    a, b, c = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    cent = (a + b + c) / 3.0
    r = cent + np.array([0.0, 0.0, 1e4])
    val = triangle_r_integral(r, a, b, c)
    assert val == pytest.approx(0.5 * 1e4, rel=1e-8)


def test_lin_grid_term_equals_dense_product():
    w = I.sphere_tiny()
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    D = lin_diagonal(o)
    Nx, Ny, Nz = o.dims
    iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) * o.h
    Hl = lin_grid_kernel(np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=-1)).real
    Pd = o.P.toarray()
    pre = np.einsum("ui,uv,vi->i", Pd, Hl, Pd)
    from oracle.lin import lin_self
    assert np.max(np.abs((lin_self(o.V, o.T) - pre) - D)) <= 1e-12 * np.max(np.abs(D))


@pytest.mark.parametrize("k", [2 * math.pi, 10.0])
def test_lin_term_improves_accuracy_against_the_direct_matrix(k):
    w = I.sphere_small()
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    D = lin_diagonal(o)
    ns = o.static_near_matrix()
    x = I.complex_gaussian(o.N, 12)
    rows = np.arange(0, o.N, 5)
    # the direct matrix with its self entries' linear term integrated exactly
    yd = dense_matvec(o.V, o.T, k, x, ns, rows) + self_lin_correction(o.V, o.T, k)[rows] * x[rows]
    e0 = np.linalg.norm(o.matvec(x, k)[rows] - yd) / np.linalg.norm(yd)
    e1 = np.linalg.norm(matvec_with_lin(o, D, x, k)[rows] - yd) / np.linalg.norm(yd)
    print(f"k={k:.2f}: AIMx {e0:.3e}, with the linear term {e1:.3e}")
    assert e1 < e0
