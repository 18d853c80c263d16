"""Pins of three oracle functions against closed forms: the Gaussian-patch
right-hand side (its integral over a sphere), iterative refinement (exact
geometric contraction under a damped inner solve, and convergence with a
single-precision inner solve), and the sphere-series density (its image
under the series operator is the plane wave; the discrete solve reproduces
it at a non-resonant wavenumber, with and without the l = 0 term)."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre

from paper_2009_02281_amd import inputs as I
from oracle import aimx, excitation, mesh, mie, solver


# -- Gaussian patch: b_i = sum_p (A_i/3) exp(-|r_ip - p|^2 / (2 sigma^2))

def gaussian_on_sphere(a, d, sigma):
    """Integral of exp(-|r - p|^2/(2 sigma^2)) over the sphere |r| = a for a
    centre p at distance d > 0 from the origin.  With |r - p|^2 =
    a^2 + d^2 - 2 a d u (u = cos of the angle to p) the surface integral is
    2 pi a^2 int_{-1}^{1} exp(-(a^2 + d^2 - 2 a d u)/(2 sigma^2)) du
    = (2 pi a sigma^2 / d) [exp(-(a-d)^2/(2 sigma^2)) - exp(-(a+d)^2/(2 sigma^2))]."""
    s2 = 2.0 * sigma * sigma
    return (2.0 * math.pi * a * sigma * sigma / d) * (math.exp(-(a - d) ** 2 / s2)
                                                     - math.exp(-(a + d) ** 2 / s2))


@pytest.mark.parametrize("d,sigma", [(0.5, 0.1), (0.5, 0.2), (0.3, 0.15), (0.8, 0.25),
                                     (0.05, 0.3)])
def test_gaussian_patch_integrates_to_closed_form(d, sigma):
    """sum_i b_i approximates the surface integral of the Gaussian on a
    radius-0.5 sphere (level-5 icosphere: flat-facet and quadrature errors
    well below 1e-3).  A factor-2 slip in the width convention, a dropped
    weight or a wrong centre changes the sum by far more than the bound."""
    V, T = I.icosphere(5, 0.5)
    rng = np.random.default_rng(11)
    u = rng.standard_normal(3)
    p = d * u / np.linalg.norm(u)
    b = excitation.gaussian_patch(V, T, p, sigma)
    exact = gaussian_on_sphere(0.5, d, sigma)
    assert b.dtype == np.complex128 and np.all(b.imag == 0)
    assert abs(b.sum().real - exact) <= 2e-3 * exact
    # the wrong width convention exp(-r^2/sigma^2) would be far off
    alt = gaussian_on_sphere(0.5, d, sigma / math.sqrt(2.0))
    assert abs(b.sum().real - alt) > 2e-2 * exact


def test_gaussian_patch_is_local_and_peaks_at_the_centre():
    """Each b_i / A_i is the mean of the Gaussian over the triangle's three
    points: it is largest on the triangle nearest the centre and matches the
    value at the centroid to second order in the mesh size."""
    V, T = I.icosphere(4, 0.5)
    c = mesh.centroids(V, T)
    A = mesh.areas(V, T)
    p = c[123] * (0.5 / np.linalg.norm(c[123]))
    sigma = 0.2
    b = excitation.gaussian_patch(V, T, p, sigma).real
    dens = b / A
    assert int(np.argmax(dens)) == 123
    at_centroid = np.exp(-np.sum((c - p) ** 2, axis=1) / (2 * sigma * sigma))
    assert np.max(np.abs(dens - at_centroid)) < 5e-3


# -- iterative refinement: x <- x + inner(b - A x)

def test_refinement_contracts_geometrically_with_a_damped_inner_solve():
    """With inner(r) = (1 - alpha) A^{-1} r the residual obeys
    r_{i+1} = alpha r_i exactly, so the recorded relative residuals are
    alpha^i and the loop stops at the first i with alpha^i <= tol."""
    rng = np.random.default_rng(3)
    n = 40
    A = np.eye(n) * 4 + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    alpha, tol = 0.3, 1e-7
    Ainv = np.linalg.inv(A)
    x, ok, hist = solver.iterative_refinement(lambda v: A @ v, lambda r: (1 - alpha) * (Ainv @ r),
                                              b, tol=tol, max_refine=50)
    steps = math.ceil(math.log(tol) / math.log(alpha))
    assert ok and len(hist) == steps + 1
    for i, h in enumerate(hist):
        assert h == pytest.approx(alpha ** i, rel=1e-6)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= tol
    # a cap below the needed count stops unconverged after max_refine steps
    x2, ok2, hist2 = solver.iterative_refinement(lambda v: A @ v,
                                                 lambda r: (1 - alpha) * (Ainv @ r), b,
                                                 tol=tol, max_refine=3)
    assert not ok2 and len(hist2) == 4 and hist2[-1] == pytest.approx(alpha ** 3, rel=1e-6)


def test_refinement_with_single_precision_inner_solve_reaches_double_accuracy():
    """Classical mixed-precision refinement (Wilkinson; Moler 1967): an inner
    solve in complex64 with unit roundoff u32 contracts the residual by
    about kappa * u32 per step, so a system with kappa ~ 1e2 reaches 1e-13 in
    a few steps although one complex64 solve alone stops near 1e-6."""
    rng = np.random.default_rng(4)
    n = 60
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A = (Q1 * np.geomspace(1.0, 1e-2, n)) @ Q2.conj().T
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A32 = A.astype(np.complex64)

    def inner(r):
        return np.linalg.solve(A32, r.astype(np.complex64)).astype(np.complex128)

    one = np.linalg.norm(b - A @ inner(b)) / np.linalg.norm(b)
    assert one > 1e-8
    x, ok, hist = solver.iterative_refinement(lambda v: A @ v, inner, b, tol=1e-13,
                                              max_refine=10)
    assert ok and len(hist) <= 6
    # contraction per step while the residual is above the float64 floor
    ratios = [hist[i + 1] / hist[i] for i in range(len(hist) - 1) if hist[i + 1] > 1e-12]
    assert ratios and max(ratios) < 1e-3
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)


# -- sphere-series density of the plane-wave problem

def test_series_density_maps_to_the_plane_wave_under_the_series_operator():
    """Project sigma(theta) from density_plane_wave onto Legendre modes with
    Gauss-Legendre quadrature, apply the series eigenvalues lam_l (pinned to
    mpmath elsewhere) and sum: the result is exp(-jka cos theta) evaluated
    directly, at a non-resonant and at a resonant-adjacent wavenumber."""
    a = 0.5
    u, wu = roots_legendre(200)
    for k in (0.9 * 2 * math.pi, 1.3 * 2 * math.pi):
        sig = mie.density_plane_wave(k, a, u)
        L = mie.lmax_for(k * a)
        ct = np.linspace(-0.95, 0.95, 13)
        img = np.zeros(ct.shape, dtype=np.complex128)
        for l in range(L + 1):
            cl = (2 * l + 1) / 2.0 * np.sum(wu * sig * eval_legendre(l, u))
            img += mie.eigenvalue(l, k, a) * cl * eval_legendre(l, ct)
        direct = np.exp(-1j * k * a * ct)
        assert np.max(np.abs(img - direct)) < 1e-10
        # dropping l = 0 removes exactly the mean of sigma over the sphere
        sig0 = mie.density_plane_wave(k, a, u, drop_l0=True)
        mean = 0.5 * np.sum(wu * sig)
        assert np.max(np.abs(sig - sig0 - mean)) < 1e-12


@pytest.mark.slow
def test_discrete_density_matches_series_at_a_non_resonant_wavenumber():
    """At k = 0.9 * 2 pi (ka = 0.45 pi, away from every zero of j_l) the AIMx
    solution of A x = b for the +z plane wave is the density itself (one
    piecewise-constant unknown per triangle).  It matches the series density
    at the centroids within discretisation error, both with the l = 0 term
    kept and with the area-weighted mean removed from both sides, and the
    error shrinks when the mesh and grid are refined (level 3, h = 0.1 ->
    level 4, h = 0.06)."""
    k = 0.9 * 2 * math.pi
    errs = []
    for lev, dims, h in [(3, (16, 16, 16), 0.1), (4, (24, 24, 24), 0.06)]:
        V, T = I.icosphere(lev, 0.5)
        o = aimx.AimOracle(V, T, 2, dims, h, 2 * h)
        b = excitation.plane_wave(V, T, k)
        x, info = solver.fgmres(lambda v: o.matvec(v, k), b, tol=1e-10, restart=60,
                                max_iter=3000)
        assert info.converged
        ct = o.cent[:, 2] / np.linalg.norm(o.cent, axis=1)
        ref = mie.density_plane_wave(k, 0.5, ct)
        A = mesh.areas(V, T)
        x0 = x - np.sum(A * x) / A.sum()
        ref0 = mie.density_plane_wave(k, 0.5, ct, drop_l0=True)
        ref0 = ref0 - np.sum(A * ref0) / A.sum()
        # the l = 0 part is not negligible here, so keeping it is a real check
        assert np.linalg.norm(ref - ref0) > 0.2 * np.linalg.norm(ref)
        errs.append((np.linalg.norm(x - ref) / np.linalg.norm(ref),
                     np.linalg.norm(x0 - ref0) / np.linalg.norm(ref0)))
    assert errs[0][0] < 0.1 and errs[0][1] < 0.1
    assert errs[1][0] < 0.7 * errs[0][0] and errs[1][1] < 0.7 * errs[0][1]
