"""Trimmed parameter space: classes, domain split and the cut-element rule.

Sect. 2.2: a B-spline is exterior, interior or cut according to the measure
of its support inside the visible domain; exterior functions leave the system.
Sect. 3, Eq. (8): the support of a cut function splits into a regular part
(elements not cut by the curve) and a trimmed part (cut elements).
Sect. 3.1: cut elements need a higher-order accurate rule; the paper uses
Lagrange sub-elements and states that any higher-order accurate scheme may
replace them.

Readings taken here:
* R5 cut rule: Gauss-Green cubature on the exact boundary of V_e = e n Omega_v.
  With a base line x0 (an element edge), int_V f = closed integral of F dy,
  F(x, y) = int_{x0}^{x} f(s, y) ds, so each boundary arc gives nodes
  (x0 + (X_q - x0)(1+tau_r)/2, Y_q) and weights
  sigma w_q dt/2 Y'(t_q) w_r (X_q - x0)/2; the visible parts of the edge
  opposite the base give a tensor Gauss rule. The horizontal bases use
  -closed integral of G dx. Of the four bases (left, right, bottom, top) the
  one with the least sum |w| is taken (first within a relative 1e-9).
  Counts: n_r = p+1 inner points, n_q = d(2p+1) points per arc of a degree-d
  curve (3 for ellipses), n_s = p+1 along straight edges; exact for c B_i B_j
  with constant c on polynomial arcs.
* Arcs: maximal pieces of a curve between grid-line crossings, curve-curve
  crossings, segment junctions and x/y extrema; an arc is kept if its midpoint
  is in the open unit square and outside every other hole. Breakpoints closer
  than 1e-13 (in the segment parameter) are merged.
* R6 classes: an element is cut iff it owns a kept arc; otherwise it is
  inside or outside by a test at its centre. A function is exterior iff all
  its support elements are outside, interior iff all are inside, else cut.
* Ordering: a cut element's nodes are its arcs in (curve, segment, t) order,
  q outer and r inner, then its visible edge segments by increasing
  coordinate, s outer and r inner.
"""
from __future__ import annotations

import math

import numpy as np

from . import bspline
from .curves import make_curve
from .quadrature import gauss

OUTSIDE, INSIDE, CUT = 0, 1, 2
EXTERIOR_FN, INTERIOR_FN, CUT_FN = 0, 1, 2
_MERGE_TOL = 1e-13


class TrimmedSpace:
    def __init__(self, patch, n_r=None, n_q=None, n_s=None):
        self.patch = patch
        self.p = p = patch.p
        self.knots1, self.knots2 = (np.asarray(k, dtype=np.float64) for k in patch.knots)
        self.bp1 = bspline.breakpoints(self.knots1, p)
        self.bp2 = bspline.breakpoints(self.knots2, p)
        self.N1, self.N2 = len(self.bp1) - 1, len(self.bp2) - 1
        self.n1, self.n2 = self.N1 + p, self.N2 + p
        self.curves = [make_curve(c) for c in patch.curves]
        self.n_r = n_r or (p + 1)
        self.n_s = n_s or (p + 1)
        self.n_q_override = n_q
        self._arcs()
        self._classify_elements()
        self._classify_functions()

    # ---------------------------------------------------------------- helpers
    def n_q(self, curve):
        if self.n_q_override:
            return self.n_q_override
        d = curve.d if curve.kind == "bspline" else 3
        return d * (2 * self.p + 1)

    def in_hole(self, x, y):
        return any(c.inside(x, y) for c in self.curves)

    def _hole_except(self, x, y, skip):
        return any(c.inside(x, y) for k, c in enumerate(self.curves) if k != skip)

    # ------------------------------------------------------------------- arcs
    def _arcs(self):
        """Arcs of the visible boundary, each inside one element."""
        arcs = []          # (curve, seg, t0, t1, e1, e2)
        for ci, c in enumerate(self.curves):
            others = []
            for cj, o in enumerate(self.curves):
                if cj == ci:
                    continue
                if c.kind == "ellipse" and o.kind == "ellipse":
                    others += c.intersect_params(o)
                else:
                    raise NotImplementedError("curve-curve crossings are only done for ellipses")
            for s in range(c.n_seg):
                lo, hi = c.seg_range(s)
                ts = [lo, hi]
                for v in self.bp1:
                    ts += c.crossings(s, 0, v)
                for v in self.bp2:
                    ts += c.crossings(s, 1, v)
                ts += c.extrema(s)
                ts += [t for t in others if lo <= t < hi]
                ts = np.sort(np.array([t for t in ts if lo <= t <= hi]))
                scale = hi - lo
                merged = [ts[0]]
                for t in ts[1:]:
                    if t - merged[-1] > _MERGE_TOL * scale:
                        merged.append(t)
                merged[-1] = hi
                if len(merged) == 1:
                    continue
                for t0, t1 in zip(merged[:-1], merged[1:]):
                    xm, ym = c.point(s, 0.5 * (t0 + t1))
                    if not (0.0 < xm < 1.0 and 0.0 < ym < 1.0):
                        continue
                    if self._hole_except(xm, ym, ci):
                        continue
                    e1 = int(bspline.element_of(self.bp1, xm))
                    e2 = int(bspline.element_of(self.bp2, ym))
                    arcs.append((ci, s, float(t0), float(t1), e1, e2))
        self.arcs = arcs
        self.arcs_of = {}
        for a in arcs:
            self.arcs_of.setdefault((a[4], a[5]), []).append(a)
        for k in self.arcs_of:
            self.arcs_of[k].sort(key=lambda a: (a[0], a[1], a[2]))

    # -------------------------------------------------------------- classes
    def _classify_elements(self):
        ecls = np.zeros((self.N2, self.N1), dtype=np.int8)
        xc = 0.5 * (self.bp1[:-1] + self.bp1[1:])
        for e2 in range(self.N2):
            yc = 0.5 * (self.bp2[e2] + self.bp2[e2 + 1])
            hole = np.zeros(self.N1, dtype=bool)
            for c in self.curves:
                hole |= c.inside_row(xc, yc)
            ecls[e2] = np.where(hole, OUTSIDE, INSIDE)
        for (e1, e2) in self.arcs_of:
            ecls[e2, e1] = CUT
        self.ecls = ecls

    def _classify_functions(self):
        p = self.p
        fcls = np.zeros((self.n2, self.n1), dtype=np.int8)
        for i2 in range(self.n2):
            for i1 in range(self.n1):
                sub = self.ecls[max(0, i2 - p):min(self.N2 - 1, i2) + 1,
                                max(0, i1 - p):min(self.N1 - 1, i1) + 1]
                if np.all(sub == OUTSIDE):
                    fcls[i2, i1] = EXTERIOR_FN
                elif np.all(sub == INSIDE):
                    fcls[i2, i1] = INTERIOR_FN
                else:
                    fcls[i2, i1] = CUT_FN
        self.fcls = fcls
        flat = fcls.reshape(-1)
        self.active = np.nonzero(flat != EXTERIOR_FN)[0]          # compact -> flat
        self.act_of = -np.ones(flat.size, dtype=np.int64)          # flat -> compact
        self.act_of[self.active] = np.arange(self.active.size)
        self.n_act = self.active.size
        # band: inside elements in the support of some cut function
        band = np.zeros_like(self.ecls, dtype=bool)
        for i2, i1 in zip(*np.nonzero(fcls == CUT_FN)):
            band[max(0, i2 - p):min(self.N2 - 1, i2) + 1, max(0, i1 - p):min(self.N1 - 1, i1) + 1] = True
        self.band = band & (self.ecls == INSIDE)

    def cut_elements(self):
        """Cut elements in flat (e2 * N1 + e1) order."""
        e2, e1 = np.nonzero(self.ecls == CUT)
        return list(zip(e1.tolist(), e2.tolist()))

    def band_elements(self):
        e2, e1 = np.nonzero(self.band)
        return list(zip(e1.tolist(), e2.tolist()))

    # -------------------------------------------------------------- cut rule
    def _line_crossings(self, axis, v, lo, hi):
        """Coordinates along the grid line {axis-coordinate = v} where curves cross it, in (lo, hi)."""
        key = (axis, float(v))
        cache = self.__dict__.setdefault("_line_cache", {})
        if key not in cache:
            allc = []
            for c in self.curves:
                for s in range(c.n_seg):
                    for t in c.crossings(s, axis, v):
                        x, y = c.point(s, t)
                        allc.append(float(y if axis == 0 else x))
            cache[key] = sorted(allc)
        return [w for w in cache[key] if lo < w < hi]

    def _visible_segments(self, axis, v, lo, hi):
        """Maximal visible sub-intervals of the edge {axis-coord = v, other in [lo, hi]}."""
        cuts = [lo] + self._line_crossings(axis, v, lo, hi) + [hi]
        segs = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            if b - a <= _MERGE_TOL * (hi - lo):
                continue
            m = 0.5 * (a + b)
            x, y = (v, m) if axis == 0 else (m, v)
            if self.in_hole(x, y):
                continue
            if segs and abs(segs[-1][1] - a) <= _MERGE_TOL * (hi - lo):
                segs[-1] = (segs[-1][0], b)
            else:
                segs.append((a, b))
        return segs

    def cut_rule(self, e1, e2, n_r=None, n_q=None, n_s=None, variant=None):
        """Nodes (x, y) and weights w of the Gauss-Green rule on V_e (the cut rule, on the exact boundary; cached)."""
        key = (e1, e2, n_r, n_q, n_s, variant)
        cache = self.__dict__.setdefault("_rule_cache", {})
        if key not in cache:
            cache[key] = self._cut_rule(e1, e2, n_r, n_q, n_s, variant)
        return cache[key]

    def _cut_rule(self, e1, e2, n_r=None, n_q=None, n_s=None, variant=None):
        n_r = n_r or self.n_r
        n_s = n_s or self.n_s
        xa, xb = self.bp1[e1], self.bp1[e1 + 1]
        ya, yb = self.bp2[e2], self.bp2[e2 + 1]
        tr, wr = gauss(n_r)
        ts_, ws_ = gauss(n_s)
        arcs = self.arcs_of.get((e1, e2), [])
        arc_data = []
        for (ci, s, t0, t1, _, _) in arcs:
            c = self.curves[ci]
            nq = n_q or self.n_q(c)
            tq, wq = gauss(nq)
            t = t0 + (t1 - t0) * (tq + 1) / 2
            wt = wq * (t1 - t0) / 2
            X, Y = c.point(s, t)
            dX, dY = c.deriv(s, t)
            arc_data.append((c.sigma, np.atleast_1d(X), np.atleast_1d(Y),
                             np.atleast_1d(dX), np.atleast_1d(dY), wt))
        # edges: (base, opposite edge segments, base coordinate, opposite coordinate)
        variants = [
            ("left", self._visible_segments(0, xb, ya, yb), xa, xb),
            ("right", self._visible_segments(0, xa, ya, yb), xb, xa),
            ("bottom", self._visible_segments(1, yb, xa, xb), ya, yb),
            ("top", self._visible_segments(1, ya, xa, xb), yb, ya),
        ]
        sums = []
        for name, segs, b0, b1 in variants:
            tot = 0.0
            for (sig, X, Y, dX, dY, wt) in arc_data:
                if name in ("left", "right"):
                    tot += np.sum(wt * np.abs(dY) * np.abs(X - b0))
                else:
                    tot += np.sum(wt * np.abs(dX) * np.abs(Y - b0))
            for (a, b) in segs:
                tot += (b - a) * abs(b1 - b0)
            sums.append(tot)
        if variant is None:
            m = min(sums)
            k = next(k for k in range(4) if sums[k] <= m * (1 + 1e-9))
        else:
            k = variant
        name, segs, b0, b1 = variants[k]
        xs, ys, ws = [], [], []
        for (sig, X, Y, dX, dY, wt) in arc_data:
            for q in range(len(X)):
                if name in ("left", "right"):
                    xs.append(b0 + (X[q] - b0) * (tr + 1) / 2)
                    ys.append(np.full(n_r, Y[q]))
                    ws.append(sig * wt[q] * dY[q] * wr * (X[q] - b0) / 2)
                else:
                    xs.append(np.full(n_r, X[q]))
                    ys.append(b0 + (Y[q] - b0) * (tr + 1) / 2)
                    ws.append(-sig * wt[q] * dX[q] * wr * (Y[q] - b0) / 2)
        for (a, b) in segs:
            for si in range(n_s):
                u = a + (b - a) * (ts_[si] + 1) / 2
                wu = ws_[si] * (b - a) / 2
                inner = b0 + (b1 - b0) * (tr + 1) / 2
                if name in ("left", "right"):
                    xs.append(inner)
                    ys.append(np.full(n_r, u))
                else:
                    xs.append(np.full(n_r, u))
                    ys.append(inner)
                ws.append(wu * wr * abs(b1 - b0) / 2)
        if not xs:
            return np.zeros(0), np.zeros(0), np.zeros(0), k
        return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws), k

    def visible_area(self):
        """Sum of the cut-rule weights plus the areas of inside elements."""
        area = 0.0
        for e2 in range(self.N2):
            for e1 in range(self.N1):
                if self.ecls[e2, e1] == INSIDE:
                    area += (self.bp1[e1 + 1] - self.bp1[e1]) * (self.bp2[e2 + 1] - self.bp2[e2])
                elif self.ecls[e2, e1] == CUT:
                    area += float(np.sum(self.cut_rule(e1, e2)[2]))
        return area
