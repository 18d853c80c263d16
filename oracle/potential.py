"""Closed-form static potential of a flat triangle (oracle).

Phi_T(r) = (1 / 4 pi) * integral over T of dS' / |r - r'|.

This is the direct integration of the frequency-independent kernel G_s
(eq. hgfs) that AIMx performs once for the near region (Sec. III-A, the
matrix L_s,NR of eq. LAIMx).  The paper delegates the singular integration
to standard singularity-extraction techniques; the closed form used here is
the classical edge-sum result (Wilton, Rao, Glisson, Schaubert, Al-Bundak
and Butler, IEEE Trans. Antennas Propag. 32(3), 1984), derived and coded
independently:

with h the signed height of r above the plane of T, rho the projection of r
on that plane and, for every edge i (endpoints p-, p+ counter-clockwise
about the normal), l+/- the signed lengths from rho's foot on the edge line
to p+/-, P0 the distance from rho to the edge line (positive inside), R0^2 =
P0^2 + h^2 and R+/- = |r - p+/-|,

  integral 1/R dS' = sum_i P0_i ln[(R+_i + l+_i) / (R-_i + l-_i)]
                     - |h| sum_i [ atan(P0_i l+_i / (R0_i^2 + |h| R+_i))
                                   - atan(P0_i l-_i / (R0_i^2 + |h| R-_i)) ].

A second routine integrates 1/R by Duffy-transformed Gauss-Legendre
quadrature; it exists only to pin the closed form.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def _log_ratio(Rp, lp, Rm, lm, R0sq):
    """ln((R+ + l+) / (R- + l-)) evaluated without cancellation: when l < 0,
    R + l is rewritten as R0^2 / (R - l)."""
    def plus(R, l):
        return R + l if l >= 0.0 else R0sq / (R - l)
    num = plus(Rp, lp)
    den = plus(Rm, lm)
    return math.log(num / den)


def triangle_inv_r(r, a, b, c) -> float:
    """Integral over triangle (a, b, c) of 1/|r - r'| dS' in closed form."""
    r = np.asarray(r, dtype=np.float64)
    verts = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    area2 = np.linalg.norm(n)
    n = n / area2
    h = float(np.dot(r - verts[0], n))
    rho = r - h * n
    ah = abs(h)
    size = math.sqrt(area2)
    total = 0.0
    for i in range(3):
        pm = verts[i]
        pp = verts[(i + 1) % 3]
        e = pp - pm
        le = np.linalg.norm(e)
        lhat = e / le
        uhat = np.cross(lhat, n)             # outward in-plane edge normal
        lp = float(np.dot(pp - rho, lhat))
        lm = float(np.dot(pm - rho, lhat))
        P0 = float(np.dot(pm - rho, uhat))   # > 0 when rho is on the inner side
        R0sq = P0 * P0 + h * h
        Rp = float(np.linalg.norm(r - pp))
        Rm = float(np.linalg.norm(r - pm))
        if abs(P0) > 1e-14 * size:
            total += P0 * _log_ratio(Rp, lp, Rm, lm, R0sq)
            if ah > 1e-14 * size:
                total -= ah * (math.atan(P0 * lp / (R0sq + ah * Rp))
                               - math.atan(P0 * lm / (R0sq + ah * Rm)))
    return total


def triangle_inv_r_points(r, a, b, c) -> np.ndarray:
    """The same closed form as ``triangle_inv_r`` for many observation
    points r[M, 3] against one triangle (array version)."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    verts = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    area2 = np.linalg.norm(n)
    n = n / area2
    size = math.sqrt(area2)
    h = (r - verts[0][None, :]) @ n
    rho = r - h[:, None] * n[None, :]
    ah = np.abs(h)
    total = np.zeros(r.shape[0])
    for i in range(3):
        pm = verts[i]
        pp = verts[(i + 1) % 3]
        e = pp - pm
        lhat = e / np.linalg.norm(e)
        uhat = np.cross(lhat, n)
        lp = (pp[None, :] - rho) @ lhat
        lm = (pm[None, :] - rho) @ lhat
        P0 = (pm[None, :] - rho) @ uhat
        R0sq = P0 * P0 + h * h
        Rp = np.linalg.norm(r - pp[None, :], axis=1)
        Rm = np.linalg.norm(r - pm[None, :], axis=1)
        use = np.abs(P0) > 1e-14 * size
        with np.errstate(divide="ignore", invalid="ignore"):
            num = np.where(lp >= 0.0, Rp + lp, R0sq / (Rp - lp))
            den = np.where(lm >= 0.0, Rm + lm, R0sq / (Rm - lm))
            logt = np.where(use, P0 * np.log(num / den), 0.0)
            att = np.arctan(P0 * lp / (R0sq + ah * Rp)) - np.arctan(P0 * lm / (R0sq + ah * Rm))
        uset = use & (ah > 1e-14 * size)
        total += logt - np.where(uset, ah * att, 0.0)
    return total


def triangle_potential(r, a, b, c) -> float:
    """Phi_T(r) = (1/4 pi) * integral of 1/R over the triangle."""
    return triangle_inv_r(r, a, b, c) / FOUR_PI


def triangle_inv_r_quadrature(r, a, b, c, order: int = 40) -> float:
    """Reference value of the same integral by numerical quadrature.

    The triangle is split at the projection rho of r into three signed
    sub-triangles (rho, v_i, v_{i+1}); on each, the Duffy map
    (u, v) -> rho + u (v_i - rho) + u v (v_{i+1} - v_i) has Jacobian
    proportional to u, which removes the 1/R singularity when r lies on the
    plane.  Gauss-Legendre with ``order`` points per direction (and per
    geometric sub-interval of u).
    """
    r = np.asarray(r, dtype=np.float64)
    A = np.asarray(a, float)
    B = np.asarray(b, float)
    C = np.asarray(c, float)
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    rho = r - np.dot(r - A, n) * n
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    # the radial variable u is split geometrically towards 0 so that points
    # just off the plane (a near-singular peak at small u) are resolved
    edges = np.concatenate([[0.0], np.logspace(-8, 0, 17)])
    ux = np.concatenate([lo + (hi - lo) * x for lo, hi in zip(edges[:-1], edges[1:])])
    uw = np.concatenate([(hi - lo) * w for lo, hi in zip(edges[:-1], edges[1:])])
    U, Vv = np.meshgrid(ux, x, indexing="ij")
    W = np.outer(uw, w)
    total = 0.0
    vs = [A, B, C]
    full2 = float(np.linalg.norm(np.cross(B - A, C - A)))
    for i in range(3):
        p1 = vs[i]
        p2 = vs[(i + 1) % 3]
        cr = np.cross(p1 - rho, p2 - rho)
        signed2 = float(np.dot(cr, n))        # twice the signed sub-area
        if abs(signed2) < 1e-13 * full2:      # rho on this edge line: no area
            continue
        pts = rho[None, None, :] + U[..., None] * (p1 - rho)[None, None, :] \
            + (U * Vv)[..., None] * (p2 - p1)[None, None, :]
        R = np.linalg.norm(pts - r[None, None, :], axis=-1)
        total += signed2 * np.sum(W * U / R)
    return total
