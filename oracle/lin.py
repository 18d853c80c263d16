"""The linear-term modification of AIMx for higher accuracy (oracle).

Sec. III-A ("Modification for Increased Accuracy", eqs. linterm and
Lmatdecomplin): the dynamic kernel G_d is not smooth at R = 0 because of its
linear Taylor term k^2 G_lin with G_lin(R) = -R / (8 pi).  The modification
treats that term separately: its entries for overlapping basis and testing
functions are integrated directly, and the grid's own contribution to those
entries is precorrected, so that

    A(k) x  ~=  C x  +  k^2 D x  +  W H(k) P x,

with C and W H(k) P as in AIMx (the grid kernel is unchanged: G_s + k^2 G_lin
+ (G - G_s - k^2 G_lin) = G for R > 0, and all three vanish or give -jk/(4 pi)
at R = 0) and, for one piecewise-constant basis function per triangle where
only a triangle overlaps itself, a real diagonal

    D_ii = A_lin[i, i] - (W H_lin P)[i, i],

A_lin[i, i] = sum_p (A_i/3) int_{T_i} G_lin(|r_ip - r'|) dS' (the 3-point
outer rule with the inner integral in closed form, the same reading as the
static near entries), H_lin the grid matrix of G_lin (0 at R = 0).

The inner integral of R over a flat triangle: in the plane of T (r at height
h above it, foot rho), div_s[(rho' - rho) R] = 3R - h^2/R, so

    int_T R dS' = (1/3) [ sum_i P0_i int_{edge i} R dl  +  h^2 int_T dS'/R ],

with P0_i the in-plane distance from rho to edge i (positive inside) and,
along edge i with foot parameter l and R0^2 = P0^2 + h^2,
int R dl = [ l R + R0^2 ln(l + R) ] / 2 between the endpoints.
"""
from __future__ import annotations

import math

import numpy as np

from . import mesh as _mesh
from .conventional import precorrection_with
from .potential import triangle_inv_r

EIGHT_PI = 8.0 * math.pi


def triangle_r_integral(r, a, b, c) -> float:
    """Integral over triangle (a, b, c) of |r - r'| dS' in closed form."""
    r = np.asarray(r, dtype=np.float64)
    verts = [np.asarray(a, float), np.asarray(b, float), np.asarray(c, float)]
    n = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    n = n / np.linalg.norm(n)
    h = float(np.dot(r - verts[0], n))
    rho = r - h * n
    edge_sum = 0.0
    for i in range(3):
        p, q = verts[i], verts[(i + 1) % 3]
        e = q - p
        L = float(np.linalg.norm(e))
        t = e / L
        m = np.cross(t, n)                       # outward in-plane edge normal
        P0 = float(np.dot(p - rho, m))
        if abs(P0) <= 1e-15 * L:
            continue
        lm = float(np.dot(p - rho, t))
        lp = float(np.dot(q - rho, t))
        R0sq = P0 * P0 + h * h
        Rm = float(np.linalg.norm(p - r))
        Rp = float(np.linalg.norm(q - r))
        # ln(l + R) between the endpoints, written without cancellation
        if lm >= 0.0:
            logs = math.log((Rp + lp) / (Rm + lm))
        elif lp <= 0.0:
            logs = math.log((Rm - lm) / (Rp - lp))
        else:
            logs = math.log((Rp + lp) * (Rm - lm) / R0sq)
        edge_sum += P0 * 0.5 * (lp * Rp - lm * Rm + R0sq * logs)
    total = edge_sum
    if h != 0.0:
        total += h * h * triangle_inv_r(r, *verts)
    return total / 3.0


def triangle_r_integral_quadrature(r, a, b, c, order: int = 60) -> float:
    """Reference value by Gauss-Legendre quadrature on a Duffy map centred at
    the projection of r (the integrand is continuous; the map resolves the
    kink of R at the foot)."""
    r = np.asarray(r, dtype=np.float64)
    A, B, C = (np.asarray(v, float) for v in (a, b, c))
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    rho = r - np.dot(r - A, n) * n
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    U, Vv = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    full2 = float(np.linalg.norm(np.cross(B - A, C - A)))
    total = 0.0
    vs = [A, B, C]
    for i in range(3):
        p1, p2 = vs[i], vs[(i + 1) % 3]
        signed2 = float(np.dot(np.cross(p1 - rho, p2 - rho), n))
        if abs(signed2) < 1e-13 * full2:
            continue
        pts = rho[None, None, :] + U[..., None] * (p1 - rho)[None, None, :] \
            + (U * Vv)[..., None] * (p2 - p1)[None, None, :]
        R = np.linalg.norm(pts - r[None, None, :], axis=-1)
        total += signed2 * np.sum(W * U * R)
    return total


def lin_self(V, T) -> np.ndarray:
    """A_lin[i, i] = sum_p (A_i/3) int_{T_i} -|r_ip - r'|/(8 pi) dS'."""
    qp = _mesh.quad_points(V, T)
    w = _mesh.quad_weights(V, T)
    out = np.empty(T.shape[0])
    for i in range(T.shape[0]):
        a, b, c = V[T[i, 0]], V[T[i, 1]], V[T[i, 2]]
        out[i] = -sum(w[i, p] * triangle_r_integral(qp[i, p], a, b, c) for p in range(3)) \
            / EIGHT_PI
    return out


def lin_grid_kernel(R):
    """G_lin on the grid: -R/(8 pi), 0 at R = 0."""
    return (-np.asarray(R, dtype=np.float64) / EIGHT_PI).astype(np.complex128)


def lin_diagonal(aim) -> np.ndarray:
    """D_ii = A_lin[i, i] - (W H_lin P)[i, i] for an AimOracle."""
    idx = np.arange(aim.N)
    pre = precorrection_with(aim.P, idx, idx, aim.dims, aim.h, lin_grid_kernel).real
    return lin_self(aim.V, aim.T) - pre


def matvec_with_lin(aim, D, x, k: float) -> np.ndarray:
    """y = C x + k^2 D x + W H(k) P x."""
    x = np.asarray(x, dtype=np.complex128)
    return aim.matvec(x, k) + (k * k) * D * x
