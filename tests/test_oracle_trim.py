"""Pins of the oracle's trimming curves, classes and cut-element rule (CPU).

Closed forms and brute force that share nothing with the oracle's cut rule:
circle areas, exact polygon clipping for straight trims (with monomial
moments integrated on triangles), adaptive 1-D quadrature of closed-form
chord lengths, and SciPy's B-spline evaluation of the trimming curve.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

from oracle import bspline
from oracle.curves import Ellipse, PeriodicBSpline
from oracle.trim import CUT, CUT_FN, EXTERIOR_FN, INSIDE, INTERIOR_FN, OUTSIDE, TrimmedSpace
from paper_2101_08053_amd import workloads as wl


# ----------------------------------------------------------------- curves
@pytest.mark.parametrize("d", [1, 2, 3])
def test_periodic_curve_matches_scipy(d):
    rng = np.random.default_rng(3)
    m = 9
    cp = rng.uniform(0, 1, size=(m, 2))
    c = PeriodicBSpline(cp, d)
    ext = np.concatenate([cp, cp[:d]], axis=0)
    knots = np.arange(m + 2 * d + 1, dtype=float)
    sx, sy = BSpline(knots, ext[:, 0], d), BSpline(knots, ext[:, 1], d)
    for s in range(m):
        t = rng.uniform(0, 1, size=5)
        x, y = c.point(s, t)
        np.testing.assert_allclose(x, sx(s + d + t), atol=1e-14)
        np.testing.assert_allclose(y, sy(s + d + t), atol=1e-14)
        dx, dy = c.deriv(s, t)
        np.testing.assert_allclose(dx, sx.derivative()(s + d + t), atol=1e-13)


def test_crossings_lie_on_lines():
    curve = wl.radial_cubic_curve(np.random.default_rng(1))
    c = PeriodicBSpline(curve.cp, 3)
    for v in np.linspace(0.2, 0.8, 13):
        for s in range(c.n_seg):
            for t in c.crossings(s, 0, v):
                assert abs(c.point(s, t)[0] - v) < 1e-14
            for t in c.crossings(s, 1, v):
                assert abs(c.point(s, t)[1] - v) < 1e-14
    e = Ellipse(0.5, 0.4, 0.2, 0.1, 0.7)
    for v in np.linspace(0.3, 0.7, 9):
        for t in e.crossings(0, 0, v):
            assert abs(e.point(0, t)[0] - v) < 1e-14


def test_circle_circle_intersection_closed_form():
    a, b = Ellipse(0.4, 0.5, 0.2, 0.2, 0.0), Ellipse(0.6, 0.5, 0.15, 0.15, 0.3)
    # circles: x-coordinate of the common chord from r1^2 - r2^2 = (x-c1)^2 - (x-c2)^2
    d = 0.2
    xr = (d * d + 0.2 ** 2 - 0.15 ** 2) / (2 * d)
    yr = math.sqrt(0.2 ** 2 - xr ** 2)
    ts = a.intersect_params(b)
    pts = sorted((round(float(a.point(0, t)[1]), 12), float(a.point(0, t)[0])) for t in ts)
    assert len(pts) == 2
    np.testing.assert_allclose([pts[0][1], pts[1][1]], [0.4 + xr] * 2, atol=1e-13)
    np.testing.assert_allclose([pts[0][0], pts[1][0]], [0.5 - yr, 0.5 + yr], atol=1e-12)


def test_orientation():
    cp = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=float)
    assert PeriodicBSpline(cp, 1).signed_area() == pytest.approx(1.0)
    assert PeriodicBSpline(cp[::-1], 1).signed_area() == pytest.approx(-1.0)


# ----------------------------------------------------------- areas: circle
@pytest.mark.parametrize("N", [8, 16, 32, 37])
def test_circle_visible_area(N):
    ts = TrimmedSpace(wl.config1(N=N))
    assert abs(ts.visible_area() - (1 - math.pi / 16)) < 1e-13


def _circle_element_area(xa, xb, ya, yb, cx=0.5, cy=0.5, r=0.25):
    """Area of [xa,xb]x[ya,yb] outside the disc, by adaptive quadrature of chord lengths."""
    def vis(x):
        dx = x - cx
        if abs(dx) >= r:
            return yb - ya
        h = math.sqrt(r * r - dx * dx)
        lo, hi = max(ya, cy - h), min(yb, cy + h)
        return (yb - ya) - max(0.0, hi - lo)
    brk = [x for x in (cx - r, cx + r) if xa < x < xb]
    val, _ = integrate.quad(vis, xa, xb, points=brk or None, epsabs=1e-15, epsrel=1e-13, limit=200)
    return val


def test_circle_element_areas_bruteforce():
    N = 12
    ts = TrimmedSpace(wl.config1(N=N))
    for (e1, e2) in ts.cut_elements():
        w = ts.cut_rule(e1, e2)[2]
        ref = _circle_element_area(ts.bp1[e1], ts.bp1[e1 + 1], ts.bp2[e2], ts.bp2[e2 + 1])
        assert abs(w.sum() - ref) < 1e-12


# ----------------------------------------------------- areas: straight line
def _clip_halfplane(poly, y0, y1):
    """Keep the part of polygon below the line through (0,y0)-(1,y1) (Sutherland-Hodgman)."""
    def f(P):
        return P[1] - (y0 + (y1 - y0) * P[0])
    out = []
    for k in range(len(poly)):
        P, Q = poly[k], poly[(k + 1) % len(poly)]
        fp, fq = f(P), f(Q)
        if fp <= 0:
            out.append(P)
        if fp * fq < 0:
            s = fp / (fp - fq)
            out.append((P[0] + s * (Q[0] - P[0]), P[1] + s * (Q[1] - P[1])))
    return out


def _poly_moment(poly, a, b):
    """int over a convex polygon of x^a y^b by a fan of collapsed (Duffy) Gauss rules."""
    if len(poly) < 3:
        return 0.0
    n = (a + b) // 2 + 3
    g, w = np.polynomial.legendre.leggauss(n)
    s, ws = (g + 1) / 2, w / 2
    tot = 0.0
    A = np.array(poly[0])
    for k in range(1, len(poly) - 1):
        B, C = np.array(poly[k]), np.array(poly[k + 1])
        J = abs((B - A)[0] * (C - B)[1] - (B - A)[1] * (C - B)[0])
        for si, wsi in zip(s, ws):
            for ti, wti in zip(s, ws):
                P = A + si * (B - A) + si * ti * (C - B)
                tot += wsi * wti * si * J * P[0] ** a * P[1] ** b
    return tot


@pytest.mark.parametrize("p", [1, 2, 4])
def test_line_trim_cut_rule_exact_moments(p):
    y0, y1 = 0.31, 0.67
    ts = TrimmedSpace(wl.table1_line(p, y0=y0, y1=y1))
    assert abs(ts.visible_area() - (1 - ((1 - y0) + (1 - y1)) / 2)) < 1e-14
    for (e1, e2) in ts.cut_elements():
        xa, xb, ya, yb = ts.bp1[e1], ts.bp1[e1 + 1], ts.bp2[e2], ts.bp2[e2 + 1]
        poly = _clip_halfplane([(xa, ya), (xb, ya), (xb, yb), (xa, yb)], y0, y1)
        x, y, w, _ = ts.cut_rule(e1, e2)
        for a in range(0, 2 * p + 1, max(1, p)):
            for b in range(0, 2 * p + 1, max(1, p)):
                ref = _poly_moment(poly, a, b)
                assert abs(np.sum(w * x ** a * y ** b) - ref) < 1e-15 + 1e-13 * abs(ref)


def test_every_base_variant_is_exact():
    ts = TrimmedSpace(wl.table1_line(3))
    for (e1, e2) in ts.cut_elements()[:4]:
        xa, xb, ya, yb = ts.bp1[e1], ts.bp1[e1 + 1], ts.bp2[e2], ts.bp2[e2 + 1]
        poly = _clip_halfplane([(xa, ya), (xb, ya), (xb, yb), (xa, yb)], 0.31, 0.67)
        for v in range(4):
            x, y, w, k = ts.cut_rule(e1, e2, variant=v)
            assert k == v
            assert abs(np.sum(w * x ** 3 * y ** 2) - _poly_moment(poly, 3, 2)) < 1e-16


# ------------------------------------------------------- areas: cubic curve
def test_cubic_hole_area_scipy():
    cfg = wl.config2(N=48)
    cp = cfg.curves[0].cp
    m, d = len(cp), 3
    ext = np.concatenate([cp, cp[:d]], axis=0)
    knots = np.arange(m + 2 * d + 1, dtype=float)
    sx, sy = BSpline(knots, ext[:, 0], d), BSpline(knots, ext[:, 1], d)
    dsy = sy.derivative()
    g, w = np.polynomial.legendre.leggauss(8)
    area = 0.0
    for s in range(m):
        u = s + d + (g + 1) / 2
        area += np.sum(w / 2 * sx(u) * dsy(u))
    ts = TrimmedSpace(cfg)
    assert abs(ts.visible_area() - (1 - abs(area))) < 1e-13


# ---------------------------------------------------- areas: ellipse union
def _union_length(x, ells, lo=0.0, hi=1.0):
    ivs = []
    for e in ells:
        # points (x, y) with implicit(x, y) < 0: quadratic in y
        cph, sph = math.cos(e.phi), math.sin(e.phi)
        dx = x - e.cx
        # u = (c dx + s dy)/a, v = (-s dx + c dy)/b -> A dy^2 + B dy + C < 0
        A = (sph / e.a) ** 2 + (cph / e.b) ** 2
        B = 2 * (cph * dx * sph / e.a ** 2 - sph * dx * cph / e.b ** 2)
        C = (cph * dx / e.a) ** 2 + (sph * dx / e.b) ** 2 - 1
        disc = B * B - 4 * A * C
        if disc > 0:
            r = math.sqrt(disc)
            ivs.append((e.cy + (-B - r) / (2 * A), e.cy + (-B + r) / (2 * A)))
    ivs.sort()
    tot, cur = 0.0, None
    for a, b in ivs:
        a, b = max(a, lo), min(b, hi)
        if b <= a:
            continue
        if cur is None or a > cur[1]:
            if cur:
                tot += cur[1] - cur[0]
            cur = [a, b]
        else:
            cur[1] = max(cur[1], b)
    if cur:
        tot += cur[1] - cur[0]
    return tot


def test_ellipse_union_area():
    cfg = wl.config3(N=40, p=3)
    ts = TrimmedSpace(cfg)
    ells = ts.curves
    brk = sorted({float(e.point(0, t)[0]) for e in ells for t in e.extrema(0)}
                 | {float(a.point(0, t)[0]) for a in ells for b in ells if a is not b for t in a.intersect_params(b)})
    brk = [x for x in brk if 0 < x < 1]
    hole, _ = integrate.quad(lambda x: _union_length(x, ells), 0, 1, points=brk, limit=400,
                             epsabs=1e-14, epsrel=1e-12)
    assert abs(ts.visible_area() - (1 - hole)) < 1e-10


# ---------------------------------------------------------------- classes
@pytest.mark.parametrize("cfg", [wl.config1(N=12), wl.config2(N=16, p=3), wl.table1_line(2)])
def test_function_classes_by_measure(cfg):
    """Classes follow |S^v_i| from the element areas: 0 -> exterior, full -> interior."""
    ts = TrimmedSpace(cfg)
    area = np.zeros((ts.N2, ts.N1))
    for e2 in range(ts.N2):
        for e1 in range(ts.N1):
            h = (ts.bp1[e1 + 1] - ts.bp1[e1]) * (ts.bp2[e2 + 1] - ts.bp2[e2])
            if ts.ecls[e2, e1] == INSIDE:
                area[e2, e1] = h
            elif ts.ecls[e2, e1] == CUT:
                area[e2, e1] = ts.cut_rule(e1, e2)[2].sum()
                assert 0 < area[e2, e1] < h
    p = ts.p
    for i2 in range(ts.n2):
        for i1 in range(ts.n1):
            sl = (slice(max(0, i2 - p), min(ts.N2 - 1, i2) + 1), slice(max(0, i1 - p), min(ts.N1 - 1, i1) + 1))
            full = sum((ts.bp1[e1 + 1] - ts.bp1[e1]) * (ts.bp2[e2 + 1] - ts.bp2[e2])
                       for e2 in range(sl[0].start, sl[0].stop) for e1 in range(sl[1].start, sl[1].stop))
            vis = area[sl].sum()
            cls = ts.fcls[i2, i1]
            if vis < 1e-15:
                assert cls == EXTERIOR_FN
            elif abs(vis - full) < 1e-15:
                assert cls == INTERIOR_FN
            else:
                assert cls == CUT_FN
