"""Writes mpmath_values.txt: arbitrary-precision reference values that pin
the oracle independently of it (this script imports mpmath only).

* G(k, r) = exp(-jkr)/(4 pi r) at a few (k, r)         -- eq. hgf
* d^m/dtheta^m of g(theta) = (exp(-j theta) - 1)/(4 pi theta) by mpmath's
  numerical differentiation at 60 digits             -- eq. Dhgf (Sec. IV-A)
* lam_l = -jk a^2 j_l(ka) h2_l(ka) (scalar sphere eigenvalues) from
  mpmath's spherical Bessel functions                 -- sphere series pin
Run: python tests/golden/make_mpmath_values.py
"""
import os

import mpmath as mp

mp.mp.dps = 60
out = []
for k, r in [(2 * mp.pi, mp.mpf("0.37")), (mp.mpf("3.1"), mp.mpf("1.9")), (mp.mpf(12), mp.mpf("0.013"))]:
    g = mp.exp(-1j * k * r) / (4 * mp.pi * r)
    out.append(f"green {mp.nstr(k, 30)} {mp.nstr(r, 30)} {mp.nstr(g.real, 25)} {mp.nstr(g.imag, 25)}")


def gfun(t):
    return (mp.exp(-1j * t) - 1) / (4 * mp.pi * t)


for m in (3, 4):
    for th in (mp.mpf("0.3"), mp.mpf("1.25"), mp.mpf("4.0")):
        d = mp.diff(gfun, th, m)
        out.append(f"dgd {m} {mp.nstr(th, 30)} {mp.nstr(d.real, 25)} {mp.nstr(d.imag, 25)}")


def sph_j(l, x):
    return mp.sqrt(mp.pi / (2 * x)) * mp.besselj(l + mp.mpf(1) / 2, x)


def sph_y(l, x):
    return mp.sqrt(mp.pi / (2 * x)) * mp.bessely(l + mp.mpf(1) / 2, x)


for ka_num, a in [(mp.mpf("0.9") * mp.pi, mp.mpf("0.5")), (2 * mp.pi * mp.mpf("0.7"), mp.mpf("0.5"))]:
    k = ka_num / a
    for l in range(4):
        x = k * a
        lam = -1j * k * a * a * sph_j(l, x) * (sph_j(l, x) - 1j * sph_y(l, x))
        out.append(f"lam {l} {mp.nstr(k, 30)} {mp.nstr(a, 30)} {mp.nstr(lam.real, 25)} {mp.nstr(lam.imag, 25)}")

path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mpmath_values.txt")
with open(path, "w") as f:
    f.write("# arbitrary-precision reference values (mpmath, 60 digits); see make_mpmath_values.py\n")
    f.write("\n".join(out) + "\n")
print(path)
