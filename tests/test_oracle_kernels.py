"""Pins of the oracle's kernel, quadrature, potential and stencil pieces
against closed forms, arbitrary-precision values and brute force."""
import math
import os

import numpy as np
import pytest

from oracle import green, mesh, potential
from oracle.aimx import lagrange_weights, stencil_start, GridError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mpmath_values.txt")


def _golden(tag):
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith(tag + " "):
                rows.append([float(v) for v in line.split()[1:]])
    return rows


# -- Green's function (Sec. II-A eq. hgf; Sec. III eqs. hgfs, hgfd, hgftaylor)

def test_green_matches_arbitrary_precision():
    for k, r, re, im in _golden("green"):
        g = complex(green.green_full(k, r))
        assert abs(g - complex(re, im)) <= 1e-15 * abs(complex(re, im))


def test_split_sums_to_full_kernel():
    rng = np.random.default_rng(1)
    r = rng.uniform(1e-3, 5.0, 200)
    k = 2 * math.pi
    full = green.green_full(k, r)
    split = green.green_static(r) + green.green_dynamic(k, r)
    assert np.max(np.abs(full - split) / np.abs(full)) < 1e-13


def test_dynamic_kernel_limit_and_taylor():
    k = 2 * math.pi
    # G_d(0) = -jk/(4 pi) (eq. hgfdtaylor, eq. Hdmm)
    assert green.green_dynamic(k, 0.0) == pytest.approx(-1j * k / (4 * math.pi), abs=1e-16)
    # continuity: tiny r approaches the limit linearly (next Taylor term)
    r = np.array([1e-6, 1e-4, 1e-2])
    gd = green.green_dynamic(k, r)
    lin = green.taylor_dynamic(k, r, 2)
    assert np.all(np.abs(gd - lin) <= 1.0 * np.abs(k ** 3 * r ** 2 / (4 * math.pi * 6)) * 1.01 + 1e-18)
    # many Taylor terms converge to the closed form at moderate r
    r = np.linspace(0.01, 0.5, 20)
    assert np.max(np.abs(green.taylor_dynamic(k, r, 40) - green.green_dynamic(k, r))) < 1e-13


def test_dynamic_kernel_is_smooth_where_static_is_singular():
    # |G_d| stays bounded by k/(4 pi) * const while G_s blows up (Sec. III)
    k = 2 * math.pi
    r = np.logspace(-12, 0, 50)
    assert np.all(np.abs(green.green_dynamic(k, r)) <= k / (4 * math.pi) * 1.0000001)


# -- interpolation error analysis (Sec. IV-A, eqs. Lbounds, Dhgf)

def test_dynamic_derivative_matches_arbitrary_precision():
    for m, th, re, im in _golden("dgd"):
        d = complex(green.dynamic_theta_derivative(th, int(m)))
        assert abs(d - complex(re, im)) <= 1e-9 * abs(complex(re, im))


def test_printed_derivative_sign_is_not_the_derivative():
    """eq. Dhgf prints (-j theta)^l; with that sign the formula misses the
    true derivative by O(1) -- the reading (+j theta)^l is the one used."""
    def printed(theta, m):
        acc = -1.0 + 0j
        for l in range(m + 1):
            acc += math.comb(m, l) * math.factorial(m - l) / math.factorial(m) \
                * (-1j * theta) ** l * np.exp(-1j * theta)
        return (-1.0) ** m * math.factorial(m) / (4 * math.pi * theta ** (m + 1)) * acc
    for m, th, re, im in _golden("dgd"):
        ref = complex(re, im)
        assert abs(printed(th, int(m)) - ref) > 1e-2 * abs(ref)


@pytest.mark.parametrize("spl", [10, 20, 30])
def test_interpolation_error_below_bound(spl):
    """Lagrange interpolation of G_d on n+1 samples at ``spl`` samples per
    wavelength stays below B_n, also inside the near region (Sec. IV-A)."""
    n = 2
    dth = 2 * math.pi / spl
    worst = 0.0
    for theta in np.linspace(0.05, 3 * math.pi, 240):
        # stencil of n+1 samples starting at the sample just below theta - dth/2
        s0 = math.floor(theta / dth - (n - 1) / 2.0)
        xs = dth * (s0 + np.arange(n + 1))
        if xs[0] <= 0:
            xs = xs - xs[0] + 1e-3 * dth   # stay on r > 0, as in the analysis
        fs = green.dynamic_theta(xs)
        err = abs(green.lagrange_interpolate(xs, fs, theta) - green.dynamic_theta(theta))
        lo, hi = min(xs[0], theta), max(xs[-1], theta)
        bound = green.interpolation_bound(lo, hi, n, samples=201)
        assert err <= bound
        worst = max(worst, err)
    # refinement reduces the error (10 -> 20 -> 30 samples per wavelength)
    assert worst < {10: 2e-3, 20: 3e-4, 30: 1e-4}[spl]


# -- the same analysis for grad G_d (Sec. IV-A, eq. Dghgf)

def test_grad_dynamic_factor_and_its_derivatives():
    """f(theta) of grad G_d = k^2 r^ f(k r) against the full gradient minus the
    static one, its limit at 0, and eq. Dghgf against arbitrary-precision
    differentiation (mpmath, 40 digits)."""
    mpmath = pytest.importorskip("mpmath")
    k = 3.7
    for r in (0.01, 0.3, 1.7):
        th = k * r
        full = -(1 + 1j * k * r) * np.exp(-1j * k * r) / (4 * math.pi * r * r)
        static = -1.0 / (4 * math.pi * r * r)
        assert k * k * complex(green.grad_dynamic_theta(th)) == pytest.approx(full - static,
                                                                               rel=1e-9)
    small = complex(green.grad_dynamic_theta(1e-3))   # -1/(8 pi) + j theta/(12 pi) + ...
    assert small.real == pytest.approx(-1 / (8 * math.pi), rel=1e-5)
    assert small.imag == pytest.approx(1e-3 / (12 * math.pi), rel=1e-2)
    mpmath.mp.dps = 40

    def f(t):
        return -((1 + 1j * t) * mpmath.exp(-1j * t) - 1) / (4 * mpmath.pi * t * t)
    for m in (1, 2, 3, 4):
        for th in (0.4, 1.3, 5.0, 11.0):
            ref = complex(mpmath.diff(f, mpmath.mpf(th), m))
            got = complex(green.grad_dynamic_theta_derivative(th, m))
            assert abs(got - ref) <= 1e-9 * abs(ref), (m, th)


@pytest.mark.parametrize("spl", [10, 20, 30])
def test_grad_interpolation_error_below_bound(spl):
    """Lagrange interpolation of grad G_d's radial factor on n+1 samples at
    ``spl`` samples per wavelength stays below B_n (eq. Dghgf in eq. Lbounds),
    also inside the near region, and shrinks with refinement (Sec. IV-A)."""
    n = 2
    dth = 2 * math.pi / spl
    worst = 0.0
    for theta in np.linspace(0.05, 3 * math.pi, 240):
        s0 = math.floor(theta / dth - (n - 1) / 2.0)
        xs = dth * (s0 + np.arange(n + 1))
        if xs[0] <= 0:
            xs = xs - xs[0] + 1e-3 * dth
        fs = green.grad_dynamic_theta(xs)
        err = abs(green.lagrange_interpolate(xs, fs, theta) - green.grad_dynamic_theta(theta))
        lo, hi = min(xs[0], theta), max(xs[-1], theta)
        assert err <= green.grad_interpolation_bound(lo, hi, n, samples=201)
        worst = max(worst, err)
    print(f"grad G_d interpolation, {spl} samples per wavelength: worst {worst:.2e}")
    assert worst < {10: 5e-4, 20: 1e-4, 30: 3e-5}[spl]


# -- quadrature

def test_three_point_rule_exact_to_degree_two():
    V = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    T = np.array([[0, 1, 2]])
    qp = mesh.quad_points(V, T)[0]
    w = mesh.quad_weights(V, T)[0]
    for a in range(3):
        for b in range(3 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * qp[:, 0] ** a * qp[:, 1] ** b)
            assert got == pytest.approx(exact, abs=1e-15)
    # and it is a degree-2 rule, not more: x^3 is not integrated exactly
    got = np.sum(w * qp[:, 0] ** 3)
    assert abs(got - 6 / 120) > 1e-4


def test_areas_and_points_inside():
    from paper_2009_02281_amd import inputs as I
    V, T = I.icosphere(2, 1.0)
    A = mesh.areas(V, T)
    # flat triangles inscribed in the unit sphere: total area below 4 pi
    assert 0.95 * 4 * math.pi < A.sum() < 4 * math.pi
    qp = mesh.quad_points(V, T)
    assert np.all(np.linalg.norm(qp, axis=-1) < 1.0)


# -- closed-form triangle potential

def test_potential_equilateral_centroid():
    s = 0.73
    a, b, c = np.array([0, 0, 0.]), np.array([s, 0, 0.]), np.array([s / 2, s * math.sqrt(3) / 2, 0])
    cen = (a + b + c) / 3
    exact = math.sqrt(3) * s * math.log(2 + math.sqrt(3))
    assert potential.triangle_inv_r(cen, a, b, c) == pytest.approx(exact, rel=1e-14)


def test_potential_far_limit():
    a, b, c = np.array([0, 0, 0.]), np.array([0.1, 0, 0.]), np.array([0.02, 0.08, 0])
    area = 0.5 * 0.1 * 0.08
    cen = (a + b + c) / 3
    for R in (10.0, 100.0):
        r = cen + R * np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81])
        got = potential.triangle_inv_r(r, a, b, c)
        assert got == pytest.approx(area / R, rel=(0.1 / R) ** 2)


def test_potential_vs_quadrature():
    rng = np.random.default_rng(3)
    for _ in range(40):
        a, b, c = rng.uniform(-1, 1, (3, 3))
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        r = rng.uniform(-1.5, 1.5, 3)
        mode = rng.integers(0, 3)
        if mode == 0:           # on the plane of the triangle
            r = r - np.dot(r - a, n) * n
        elif mode == 1:         # on an edge line
            t = rng.uniform(-1, 2)
            r = a + t * (b - a)
        exact = potential.triangle_inv_r(r, a, b, c)
        ref = potential.triangle_inv_r_quadrature(r, a, b, c, order=160)
        assert exact == pytest.approx(ref, rel=1e-10)
        vec = potential.triangle_inv_r_points(r[None, :], a, b, c)[0]
        assert vec == pytest.approx(exact, rel=1e-13)


# -- stencils (moment matching, Sec. IV: equivalent to interpolation)

@pytest.mark.parametrize("order", [2, 3])
def test_lagrange_reproduces_polynomials(order):
    rng = np.random.default_rng(order)
    u = rng.uniform((order - 1) / 2, (order + 1) / 2, 50)
    L = lagrange_weights(u, order)
    nodes = np.arange(order + 1)
    assert np.allclose(L.sum(axis=-1), 1.0, atol=1e-14)
    for p in range(order + 1):
        assert np.allclose(L @ nodes ** p, u ** p, rtol=0, atol=1e-12)
    # degree n+1 is not reproduced
    assert not np.allclose(L @ nodes ** (order + 1), u ** (order + 1), atol=1e-6)


@pytest.mark.parametrize("order", [2, 3])
def test_stencil_start_symmetric_and_bounded(order):
    rng = np.random.default_rng(10 + order)
    origin = np.array([-1.0, -2.0, 0.5])
    h = 0.1
    dims = (20, 20, 20)
    pts = origin + h * rng.uniform(3, 15, (100, 3))
    s, u = stencil_start(pts, origin, h, order, dims)
    assert np.all(u >= (order - 1) / 2 - 1e-12) and np.all(u < (order + 1) / 2 + 1e-12)
    with pytest.raises(GridError):
        stencil_start(origin[None, :] + h * 0.2, origin, h, order, dims)
