"""Helmholtz Green's function and the AIMx kernel split (oracle).

Follows Sec. II-A (eq. hgf) and Sec. III (eqs. hgftaylor, hgfdecomp0, hgfs,
hgfd, hgfdtaylor) with the e^{j omega t} time convention, so the outgoing
kernel is e^{-jkr}/(4 pi r).  Also the Lagrange-interpolation error bound of
Sec. IV-A (eq. Lbounds) with the (n+1)-th derivative of G_d (eq. Dhgf), in
the corrected reading documented below.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def green_full(k: float, r):
    """G(k, r) = exp(-j k r) / (4 pi r)  (eq. hgf); r > 0."""
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-1j * k * r) / (FOUR_PI * r)


def green_static(r):
    """G_s(r) = 1 / (4 pi r)  (eq. hgfs); r > 0."""
    r = np.asarray(r, dtype=np.float64)
    return 1.0 / (FOUR_PI * r)


def green_dynamic(k: float, r):
    """G_d(k, r) = (exp(-j k r) - 1) / (4 pi r)  (eq. hgfd).

    Evaluated through exp(-jx) - 1 = -2 sin^2(x/2) - j sin(x), which has no
    cancellation for small x.  At r = 0 it takes its limit -jk/(4 pi), the
    first term of the Taylor series (eq. hgfdtaylor).
    """
    r = np.asarray(r, dtype=np.float64)
    out = np.empty(r.shape, dtype=np.complex128)
    zero = r == 0.0
    rz = np.where(zero, 1.0, r)
    x = k * rz
    s = np.sin(0.5 * x)
    val = (-2.0 * s * s - 1j * np.sin(x)) / (FOUR_PI * rz)
    out[...] = np.where(zero, -1j * k / FOUR_PI, val)
    return out


def taylor_dynamic(k: float, r, terms: int):
    """Partial sum of eq. hgfdtaylor: sum_{m=1}^{terms} (-jk)^m r^{m-1} / (4 pi m!)."""
    r = np.asarray(r, dtype=np.float64)
    acc = np.zeros(r.shape, dtype=np.complex128)
    for m in range(1, terms + 1):
        acc = acc + (-1j * k) ** m * r ** (m - 1) / (FOUR_PI * math.factorial(m))
    return acc


def dynamic_theta(theta):
    """g(theta) = (exp(-j theta) - 1) / (4 pi theta): G_d in the normalised
    coordinate theta = k r of Sec. IV-A, so that G_d(k, r) = k g(k r)."""
    theta = np.asarray(theta, dtype=np.float64)
    return green_dynamic(1.0, theta)


def dynamic_theta_derivative(theta, m: int):
    """m-th derivative of g(theta) = (exp(-j theta) - 1)/(4 pi theta).

    Leibniz' rule on f(theta) * theta^{-1} with f = exp(-j theta) - 1 gives

        g^(m) = (-1)^m m! / (4 pi theta^{m+1}) *
                [ -1 + sum_{l=0}^{m} C(m,l) (m-l)!/m! (+j theta)^l e^{-j theta} ].

    This is eq. Dhgf with m = n+1 except for the sign inside the power: the
    printed form has (-j theta)^l, which does not equal the derivative
    (reading recorded in the design notes; the tests check this form against
    arbitrary-precision differentiation).
    """
    theta = np.asarray(theta, dtype=np.float64)
    acc = np.full(theta.shape, -1.0 + 0j)
    e = np.exp(-1j * theta)
    for l in range(m + 1):
        acc = acc + math.comb(m, l) * math.factorial(m - l) / math.factorial(m) \
            * (1j * theta) ** l * e
    return (-1.0) ** m * math.factorial(m) / (FOUR_PI * theta ** (m + 1)) * acc


def interpolation_bound(theta0: float, thetan: float, n: int, samples: int = 2001):
    """B_n of eq. Lbounds for K = G_d: (theta_n - theta_0)^{n+1}/(n+1)! times
    the largest |g^{(n+1)}| on [theta_0, theta_n] (maximum taken on a dense
    sample of the interval)."""
    xi = np.linspace(theta0, thetan, samples)
    dmax = np.max(np.abs(dynamic_theta_derivative(xi, n + 1)))
    return (thetan - theta0) ** (n + 1) / math.factorial(n + 1) * dmax


def grad_dynamic_theta(theta):
    """The radial factor of grad G_d in the normalised coordinate theta = k r:
    grad G_d(k, r) = k^2 r^ f(theta), f(theta) = -[(1 + j theta) e^{-j theta} - 1]
    / (4 pi theta^2) (eqs. ghgf and ghgfd); its limit at 0 is -1/(8 pi)."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.empty(theta.shape, dtype=np.complex128)
    zero = theta == 0.0
    t = np.where(zero, 1.0, theta)
    val = -((1.0 + 1j * t) * np.exp(-1j * t) - 1.0) / (FOUR_PI * t * t)
    out[...] = np.where(zero, -1.0 / (2.0 * FOUR_PI), val)
    return out


def grad_dynamic_theta_derivative(theta, m: int):
    """m-th derivative of f (eq. Dghgf with m = n+1): Leibniz' rule on
    u(theta) theta^{-2} with u = (1 + j theta) e^{-j theta} - 1, whose l-th
    derivative is -delta_l + (-j)^l e^{-j theta} (1 + j theta - l), and
    (theta^{-2})^{(m-l)} = (-m-1+l)_{m-l} theta^{-(m+2-l)} (Pochhammer)."""
    theta = np.asarray(theta, dtype=np.float64)
    e = np.exp(-1j * theta)
    acc = np.zeros(theta.shape, dtype=np.complex128)
    for l in range(m + 1):
        a, poch = -m - 1 + l, 1.0
        for i in range(m - l):
            poch *= a + i
        ul = (-1j) ** l * e * (1.0 + 1j * theta - l) - (1.0 if l == 0 else 0.0)
        acc = acc + math.comb(m, l) * poch / theta ** (m + 2 - l) * ul
    return -acc / FOUR_PI


def grad_interpolation_bound(theta0: float, thetan: float, n: int, samples: int = 2001):
    """B_n of eq. Lbounds for the radial factor of grad G_d."""
    xi = np.linspace(theta0, thetan, samples)
    dmax = np.max(np.abs(grad_dynamic_theta_derivative(xi, n + 1)))
    return (thetan - theta0) ** (n + 1) / math.factorial(n + 1) * dmax


def lagrange_interpolate(xs, fs, x):
    """Lagrange polynomial through (xs[q], fs[q]) evaluated at x
    (the interpolant of Sec. IV-A)."""
    xs = np.asarray(xs, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.complex128)
    for q in range(xs.size):
        basis = np.ones(x.shape)
        for m in range(xs.size):
            if m != q:
                basis = basis * (x - xs[m]) / (xs[q] - xs[m])
        out = out + fs[q] * basis
    return out
