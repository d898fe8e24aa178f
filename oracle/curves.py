"""Trimming curves in the parameter space (Sect. 2.2).

A trimming curve is closed and bounds one hole; the visible domain is the
unit square minus the union of the holes. The paper leaves the curve
representation open; two kinds are taken here:

* ``PeriodicBSpline`` -- closed uniform B-spline of degree 1..3 (a polygon for
  degree 1); segment k runs over t in [0, 1] and uses control points
  P_k .. P_{k+d} (indices mod m). Its blending polynomials are obtained by
  interpolating the cardinal B-spline (evaluated by the B-spline recursion)
  at d+1 points.
* ``Ellipse`` -- exact trigonometric parametrisation, one segment t in [0, 2 pi).

Each kind offers: point and derivative, crossings with a grid line (a root
finder of NumPy or a closed form), extrema parameters (roots of X' and Y'),
an inside test, and its orientation.
"""
from __future__ import annotations

import math

import numpy as np

from . import bspline

_ROOT_IMAG_TOL = 1e-7


def _real_roots_in(coeffs_high_first, lo, hi, poly_eval=None, deriv_eval=None):
    """Real roots in [lo, hi) of a polynomial, polished by Newton steps."""
    c = np.trim_zeros(np.asarray(coeffs_high_first, dtype=np.float64), "f")
    if len(c) <= 1:
        return []
    r = np.roots(c)
    out = []
    dc = np.polyder(c)
    for z in r:
        if abs(z.imag) > _ROOT_IMAG_TOL * (1.0 + abs(z.real)):
            continue
        t = z.real
        for _ in range(4):
            d = np.polyval(dc, t)
            if d == 0.0:
                break
            step = np.polyval(c, t) / d
            t -= step
            if abs(step) < 1e-18:
                break
        if lo - 1e-14 <= t < hi:
            out.append(min(max(t, lo), hi))
    return sorted(out)


class PeriodicBSpline:
    kind = "bspline"

    def __init__(self, cp, degree):
        self.cp = np.asarray(cp, dtype=np.float64)
        self.d = int(degree)
        self.m = len(self.cp)
        assert 1 <= self.d <= 3 and self.m > self.d
        self.blend = self._blending(self.d)          # (d+1, d+1): row l = coeffs (high first) of N_l(t)
        self.px, self.py = [], []
        for k in range(self.m):
            P = self.cp[[(k + l) % self.m for l in range(self.d + 1)]]
            self.px.append(self.blend.T @ P[:, 0])     # coefficient array, high power first
            self.py.append(self.blend.T @ P[:, 1])
        self.n_seg = self.m
        self.sigma = -1.0 if self.signed_area() > 0 else 1.0

    @staticmethod
    def _blending(d):
        """Blending polynomials of the uniform B-spline of degree d on one unit span.

        Knots 0..2d+1; on span [d, d+1] the non-zero functions are B_0..B_d
        (B_l has support [l, l+d+1]). Interpolating their values at d+1 points
        gives their exact polynomial coefficients in t = u - d.
        """
        knots = np.arange(2 * d + 2, dtype=np.float64)
        ts = np.linspace(0.0, 1.0, d + 1) if d > 0 else np.array([0.5])
        rows = []
        for l in range(d + 1):
            vals = bspline._basis_recursive(knots, d, l, d + ts, d)
            rows.append(np.polyfit(ts, vals, d))
        return np.array(rows)

    def seg_range(self, s):
        return 0.0, 1.0

    def point(self, s, t):
        return np.polyval(self.px[s], t), np.polyval(self.py[s], t)

    def deriv(self, s, t):
        return np.polyval(np.polyder(self.px[s]), t), np.polyval(np.polyder(self.py[s]), t)

    def crossings(self, s, axis, c):
        poly = (self.px[s] if axis == 0 else self.py[s]).copy()
        poly[-1] -= c
        return _real_roots_in(poly, 0.0, 1.0)

    def extrema(self, s):
        out = []
        for poly in (self.px[s], self.py[s]):
            out += [t for t in _real_roots_in(np.polyder(poly), 0.0, 1.0) if 0.0 < t < 1.0]
        return out

    def signed_area(self):
        """(1/2) closed integral of (x dy - y dx), exact by Gauss on each polynomial segment."""
        tg, wg = np.polynomial.legendre.leggauss(2 * self.d + 2)
        t, w = (tg + 1) / 2, wg / 2
        A = 0.0
        for s in range(self.m):
            x, y = self.point(s, t)
            dx, dy = self.deriv(s, t)
            A += 0.5 * np.sum(w * (x * dy - y * dx))
        return A

    def row_crossings(self, y):
        """x-coordinates where the curve crosses the horizontal line at height y."""
        out = []
        for s in range(self.m):
            for t in self.crossings(s, 1, y):
                out.append(float(self.point(s, t)[0]))
        return np.array(out)

    def inside(self, x, y):
        """Even-odd count of crossings of the ray {(s, y): s > x} with the curve."""
        xc = self.row_crossings(y)
        return np.sum(xc > x) % 2 == 1

    def inside_row(self, xs, y):
        xc = self.row_crossings(y)
        return (np.sum(xc[None, :] > np.asarray(xs)[:, None], axis=1) % 2) == 1


class Ellipse:
    kind = "ellipse"

    def __init__(self, cx, cy, a, b, phi):
        self.cx, self.cy, self.a, self.b, self.phi = map(float, (cx, cy, a, b, phi))
        cph, sph = math.cos(self.phi), math.sin(self.phi)
        # X = cx + A1 cos t + A2 sin t, Y = cy + C1 cos t + C2 sin t
        self.A1, self.A2 = self.a * cph, -self.b * sph
        self.C1, self.C2 = self.a * sph, self.b * cph
        self.n_seg = 1
        self.sigma = -1.0          # counter-clockwise: the hole is traversed backwards

    def seg_range(self, s):
        return 0.0, 2.0 * math.pi

    def point(self, s, t):
        return (self.cx + self.A1 * np.cos(t) + self.A2 * np.sin(t),
                self.cy + self.C1 * np.cos(t) + self.C2 * np.sin(t))

    def deriv(self, s, t):
        return (-self.A1 * np.sin(t) + self.A2 * np.cos(t),
                -self.C1 * np.sin(t) + self.C2 * np.cos(t))

    def crossings(self, s, axis, c):
        P, Q, c0 = (self.A1, self.A2, self.cx) if axis == 0 else (self.C1, self.C2, self.cy)
        R = math.hypot(P, Q)
        v = (c - c0) / R
        if abs(v) > 1.0:
            return []
        d = math.atan2(Q, P)
        ac = math.acos(v)
        out = sorted({(d + ac) % (2 * math.pi), (d - ac) % (2 * math.pi)})
        return out

    def extrema(self, s):
        out = []
        for P, Q in ((self.A1, self.A2), (self.C1, self.C2)):
            d = math.atan2(Q, P)             # derivative -P sin t + Q cos t = 0 at t = d, d + pi
            out += [d % (2 * math.pi), (d + math.pi) % (2 * math.pi)]
        return out

    def implicit(self, x, y):
        cph, sph = math.cos(self.phi), math.sin(self.phi)
        dx, dy = x - self.cx, y - self.cy
        u = (cph * dx + sph * dy) / self.a
        v = (-sph * dx + cph * dy) / self.b
        return u * u + v * v - 1.0

    def inside(self, x, y):
        return self.implicit(x, y) < 0.0

    def inside_row(self, xs, y):
        return self.implicit(np.asarray(xs), y) < 0.0

    def intersect_params(self, other):
        """Parameters t of this ellipse where it meets ellipse ``other``.

        g_other(P(t)) is a quadratic in (cos t, sin t); with s = tan(t/2) it
        becomes a quartic in s whose real roots give the crossings.
        """
        cph, sph = math.cos(other.phi), math.sin(other.phi)
        d0 = (self.cx - other.cx, self.cy - other.cy)

        def proj(ux, uy):
            return (ux * d0[0] + uy * d0[1], ux * self.A1 + uy * self.C1, ux * self.A2 + uy * self.C2)

        U0, U1, U2 = proj(cph, sph)
        V0, V1, V2 = proj(-sph, cph)
        # (1+s^2) * (U0 + U1 cos + U2 sin) = (U0 - U1) s^2 + 2 U2 s + (U0 + U1)
        Ut = np.array([U0 - U1, 2 * U2, U0 + U1]) / other.a
        Vt = np.array([V0 - V1, 2 * V2, V0 + V1]) / other.b
        poly = np.polymul(Ut, Ut) + np.polymul(Vt, Vt) - np.polymul([1, 0, 1], [1, 0, 1])
        out = []
        for z in np.roots(np.trim_zeros(poly, "f")):
            if abs(z.imag) > 1e-6 * (1 + abs(z.real)):
                continue
            t = 2.0 * math.atan(z.real)
            for _ in range(6):                       # Newton on g_other(P(t))
                x, y = self.point(0, t)
                dx, dy = self.deriv(0, t)
                gx = 2 * ((cph * (x - other.cx) + sph * (y - other.cy)) * cph / other.a ** 2
                          - (-sph * (x - other.cx) + cph * (y - other.cy)) * sph / other.b ** 2)
                gy = 2 * ((cph * (x - other.cx) + sph * (y - other.cy)) * sph / other.a ** 2
                          + (-sph * (x - other.cx) + cph * (y - other.cy)) * cph / other.b ** 2)
                der = gx * dx + gy * dy
                if der == 0:
                    break
                t -= other.implicit(x, y) / der
            x, y = self.point(0, t)
            if abs(other.implicit(x, y)) < 1e-10:
                out.append(t % (2 * math.pi))
        return sorted(out)


def make_curve(c):
    from paper_2101_08053_amd import workloads as wl
    if c.kind == wl.CURVE_BSPLINE:
        return PeriodicBSpline(c.cp, c.degree)
    if c.kind == wl.CURVE_ELLIPSE:
        return Ellipse(c.cx, c.cy, c.a, c.b, c.phi)
    raise ValueError("unknown curve kind")
