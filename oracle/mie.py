"""Scalar single-layer series on a sphere ("Mie" pin) -- oracle.

Not printed in the paper (which compares its vector EFIE with the Mie
series, Sec. IV-C); this is the scalar analogue from the spherical addition
theorem for the e^{-jkR}/(4 pi R) kernel (e^{j omega t} convention):

  e^{-jkR}/(4 pi R) = -jk sum_l (2l+1)/(4 pi) j_l(k r<) h2_l(k r>) P_l(cos g)

with h2_l = j_l - j y_l.  On a sphere of radius a the single-layer operator
S is diagonal in Legendre modes: S[P_l(cos th)] = lam_l P_l(cos th),
lam_l = -jk a^2 j_l(ka) h2_l(ka).  A plane wave along +z expands as
exp(-jkz) = sum_l (-j)^l (2l+1) j_l(kr) P_l(cos th); the density solving
S sigma = u_inc and its exterior field follow mode by mode.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def h2(l, x):
    return spherical_jn(l, x) - 1j * spherical_yn(l, x)


def lmax_for(ka: float) -> int:
    return int(ka + 4.0 * ka ** (1.0 / 3.0) + 12)


def green_series(k: float, r1: float, r2: float, cosg: float, lmax: int | None = None):
    """The addition-theorem series for G between points at radii r1, r2
    separated by angle acos(cosg)."""
    rl, rg = min(r1, r2), max(r1, r2)
    L = lmax_for(k * rg) + 20 if lmax is None else lmax
    s = 0j
    for l in range(L + 1):
        s += (2 * l + 1) / (4 * math.pi) * spherical_jn(l, k * rl) * h2(l, k * rg) \
            * eval_legendre(l, cosg)
    return -1j * k * s


def eigenvalue(l: int, k: float, a: float) -> complex:
    """lam_l = -jk a^2 j_l(ka) h2_l(ka)."""
    return -1j * k * a * a * spherical_jn(l, k * a) * h2(l, k * a)


def density_plane_wave(k: float, a: float, cos_theta, drop_l0: bool = False):
    """sigma(theta) solving S sigma = exp(-jkz) on the sphere:
    sum_l (-j)^l (2l+1) P_l(cos th) / (-jk a^2 h2_l(ka)).
    With ``drop_l0`` the (possibly undetermined) l = 0 term is left out."""
    ct = np.asarray(cos_theta, dtype=np.float64)
    out = np.zeros(ct.shape, dtype=np.complex128)
    for l in range(0 if not drop_l0 else 1, lmax_for(k * a) + 1):
        out += (-1j) ** l * (2 * l + 1) * eval_legendre(l, ct) / (-1j * k * a * a * h2(l, k * a))
    return out


def exterior_field_plane_wave(k: float, a: float, r, cos_theta):
    """Field radiated by that density at radius r >= a:
    sum_l (-j)^l (2l+1) j_l(ka) h2_l(kr)/h2_l(ka) P_l(cos th)."""
    ct = np.asarray(cos_theta, dtype=np.float64)
    out = np.zeros(ct.shape, dtype=np.complex128)
    for l in range(lmax_for(k * r) + 1):
        out += (-1j) ** l * (2 * l + 1) * spherical_jn(l, k * a) * h2(l, k * r) / h2(l, k * a) \
            * eval_legendre(l, ct)
    return out
