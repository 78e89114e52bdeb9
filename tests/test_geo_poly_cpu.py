"""Host-side check of the squared-geodesic polynomials the sphere pair loops
use (Sec. 6.4 cost): the coefficient table of the header, evaluated by
Horner's rule in FP64 as the kernels do, against asin/acos from the C
library, on the near branch (squared chord s <= 2) and through the antipode
on the far branch."""
import math
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2507_23602_amd", "csrc", "rsot_geo_poly.h")


def _coeffs(name="geo"):
    txt = open(HEADER).read()
    out = {}
    for deg, body in re.findall(r"rsot_" + name + r"_poly(\d+)\[\d+\] = \{(.*?)\};", txt,
                                flags=re.S):
        out[int(deg)] = [float(v) for v in body.replace("\n", " ").split(",")]
    return out


def _F(c, v):
    f = c[-1]
    for ci in c[-2::-1]:
        f = f * v + ci
    return f


def _geo2(c, x, y):
    """the kernels' formula, scalar FP64: squared chord s = 2 - 2 x.y, the
    polynomial on the near hemisphere, the antipode's chord u = 4 - s on the
    far one"""
    s = 2.0 - 2.0 * float(x @ y)
    if s <= 2.0:
        return s * _F(c, s)
    u = max(4.0 - s, 0.0)
    return (math.pi - math.sqrt(u * _F(c, u))) ** 2


def test_tables_have_the_stated_degrees_and_start_at_one():
    c = _coeffs()
    assert sorted(c) == [14, 18]
    assert len(c[14]) == 15 and len(c[18]) == 19
    # F(0) = 1 and F'(0) = 1/12 (the series 1 + v/12 + v^2/90 + ...)
    assert abs(c[18][0] - 1.0) < 1e-15 and abs(c[18][1] - 1.0 / 12.0) < 1e-12
    assert abs(c[18][2] - 1.0 / 90.0) < 1e-10


def test_near_branch_against_asin():
    c = _coeffs()
    for deg, tol in ((14, 3e-13), (18, 2e-15)):
        worst = 0.0
        for s in np.linspace(0.0, 2.0, 2001):
            g = (2.0 * math.asin(math.sqrt(s) / 2.0)) ** 2
            worst = max(worst, abs(s * _F(c[deg], s) - g))
        assert worst < tol, (deg, worst)


def test_pairs_against_acos_on_both_hemispheres():
    c = _coeffs()
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4000, 3))
    y = rng.standard_normal((4000, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    # include near-coincident and near-antipodal pairs
    y[:200] = x[:200] + 1e-4 * rng.standard_normal((200, 3))
    y[200:400] = -x[200:400] + 1e-4 * rng.standard_normal((200, 3))
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    far = 0
    for deg, tol in ((14, 1e-12), (18, 1e-14)):
        worst = 0.0
        for a, b in zip(x, y):
            # the reference distance from the cross and dot products (well
            # conditioned everywhere, unlike acos alone near +-1); the dot
            # product's rounding (a few 1e-16) moves d_g by that over the
            # antipode's chord |a + b|, as it moves acos near -1
            ref = math.atan2(float(np.linalg.norm(np.cross(a, b))), float(a @ b)) ** 2
            u = float(np.sum((a + b) ** 2))
            cond = 2.0 * math.pi * 1e-15 / math.sqrt(u) if u < 2.0 else 0.0
            worst = max(worst, abs(_geo2(c[deg], a, b) - ref) - cond)
            far += u < 2.0
        assert worst < tol, (deg, worst)
    assert far > 3000                     # both branches exercised


def test_log_map_factor_against_sin():
    """theta / sin(theta) of the logarithmic map from the squared chord, on
    the near hemisphere (s <= 2), against asin and sin; H(0) = 1 and
    H(2) = pi / 2."""
    c = _coeffs("logmap")
    assert sorted(c) == [16, 20]
    for deg, tol in ((16, 1e-13), (20, 2e-15)):
        assert abs(_F(c[deg], 0.0) - 1.0) < tol
        assert abs(_F(c[deg], 2.0) - math.pi / 2.0) < tol
        worst = 0.0
        for s in np.linspace(1e-6, 2.0, 2001):
            th = 2.0 * math.asin(math.sqrt(s) / 2.0)
            worst = max(worst, abs(_F(c[deg], s) - th / math.sin(th)))
        assert worst < tol, (deg, worst)
