"""Input generators: the resonance screens used by the batch of uneven
geometries, and the batch itself."""
import math

import pytest
from scipy.special import spherical_jn

from paper_2009_02281_amd import inputs as I


def test_sphere_margin_vanishes_at_zeros_of_spherical_bessel():
    # ka = pi is a zero of j_0; 16.6411 is near a zero of j_8
    assert abs(spherical_jn(0, math.pi)) < 1e-15
    assert I.sphere_resonance_margin(math.pi) < 1e-12
    assert I.sphere_resonance_margin(16.6411) < 0.01
    # half way between zeros the margin is of order one
    assert I.sphere_resonance_margin(0.75 * math.pi) > 0.1


def test_box_gap_vanishes_on_a_cavity_mode():
    a, b, c = 1.0, 1.3, 2.1
    k = math.pi * math.sqrt(1 / a ** 2 + 2 ** 2 / b ** 2 + 1 / c ** 2)
    assert I.box_resonance_gap(k, (a, b, c)) < 1e-12
    assert I.box_resonance_gap(k * 1.001, (a, b, c)) > 0.0


def test_uneven_batch_avoids_resonances_and_spans_sizes():
    ws = I.uneven_batch()
    assert len(ws) == 32
    ns = [w.n for w in ws]
    assert min(ns) >= 5000 and max(ns) <= 120000
    for w in ws:
        lam = 2 * math.pi / float(w.k[0])
        assert lam / 12 - 1e-12 <= w.extra["edge"] <= lam / 8 + 1e-12
        if w.extra["kind"].startswith("sphere"):
            a = float(abs(w.vertices).max())
            assert I.sphere_resonance_margin(float(w.k[0]) * a) >= 0.15
    assert {w.extra["kind"].split("-")[0] for w in ws} == {"sphere", "box", "boxarray"}
