"""Pins of the oracle's formation (Eqs. (6)-(7), Sects. 3.2 and 4.1) on the CPU."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import bspline
from oracle.assemble import Oracle, from_ell, to_ell
from oracle.geometry import Coefficient, map_and_detj
from oracle.trim import INTERIOR_FN
from paper_2101_08053_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_massmatrix_error.json")


def _const(cfg):
    return Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_CONST))


CASES = [wl.config1(N=12), wl.config2(N=14, p=3), wl.config3(N=16, p=2), wl.table1_line(3),
         wl.nonuniform_variant(wl.config1(N=12, p=3)), wl.nonuniform_variant(wl.config2(N=10, p=4))]


@pytest.mark.parametrize("cfg", CASES, ids=lambda c: c.name)
def test_c1_invariants(cfg):
    o = _const(cfg)
    G = o.gauss_reference()
    H = o.hybrid()
    Gd = G.toarray()
    scale = np.abs(Gd).max()
    assert np.abs(Gd - Gd.T).max() <= 1e-14 * scale
    area = o.ts.visible_area()
    assert abs(G.sum() - area) < 1e-13
    assert abs(H.sum() - area) < 1e-13
    assert np.abs((H - G).toarray()).max() <= 1e-13 * scale
    # row sums of interior rows: int B_i = prod_d (xi_{i+p+1} - xi_i)/(p+1)
    p = cfg.p
    k1, k2 = o.ts.knots1, o.ts.knots2
    rs = np.asarray(H.sum(axis=1)).ravel()
    for f in np.nonzero(o.ts.fcls.reshape(-1) == INTERIOR_FN)[0][::7]:
        i2, i1 = divmod(int(f), o.ts.n1)
        ref = (k1[i1 + p + 1] - k1[i1]) / (p + 1) * (k2[i2 + p + 1] - k2[i2]) / (p + 1)
        assert abs(rs[o.ts.act_of[f]] - ref) < 1e-15


def test_table1_magnitudes():
    """Hybrid Gauss agrees with element Gauss at round-off; naive WQ does not (Table 1)."""
    gold = json.load(open(GOLDEN))["rows"]
    for p in range(1, 7):
        o = _const(wl.table1_line(p))
        G = o.gauss_reference().toarray()
        eh = np.linalg.norm(o.hybrid().toarray() - G)
        en = np.linalg.norm(o.naive().toarray() - G)
        hyb_paper, _, naive_paper = gold[str(p)]
        assert eh <= max(hyb_paper, 1e-16) * 10
        assert naive_paper / 5 <= en <= naive_paper * 5


def _clip_below(poly, y0, y1):
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


def test_line_trim_matrix_bruteforce():
    """M (c = 1) against polygon clipping plus collapsed-Gauss integration of B_i B_j."""
    p, N, y0, y1 = 2, 5, 0.31, 0.67
    cfg = wl.table1_line(p, N=N, y0=y0, y1=y1)
    o = _const(cfg)
    G = o.gauss_reference().toarray()
    ts = o.ts
    k1, k2 = ts.knots1, ts.knots2
    n = 6
    g, w = np.polynomial.legendre.leggauss(n)
    s, ws = (g + 1) / 2, w / 2
    ref = np.zeros_like(G)
    for e2 in range(N):
        for e1 in range(N):
            xa, xb, ya, yb = ts.bp1[e1], ts.bp1[e1 + 1], ts.bp2[e2], ts.bp2[e2 + 1]
            poly = _clip_below([(xa, ya), (xb, ya), (xb, yb), (xa, yb)], y0, y1)
            if len(poly) < 3:
                continue
            A = np.array(poly[0])
            for k in range(1, len(poly) - 1):
                B, C = np.array(poly[k]), np.array(poly[k + 1])
                J = abs((B - A)[0] * (C - B)[1] - (B - A)[1] * (C - B)[0])
                S, T = np.meshgrid(s, s, indexing="ij")
                WW = np.outer(ws, ws) * S * J
                P = A[None, None, :] + S[..., None] * (B - A) + (S * T)[..., None] * (C - B)
                x, y, wt = P[..., 0].ravel(), P[..., 1].ravel(), WW.ravel()
                B1 = bspline.local_basis(k1, p, e1, x)
                B2 = bspline.local_basis(k2, p, e2, y)
                for a2 in range(p + 1):
                    for a1 in range(p + 1):
                        fa = ts.act_of[(e2 + a2) * ts.n1 + e1 + a1]
                        for b2 in range(p + 1):
                            for b1 in range(p + 1):
                                fb = ts.act_of[(e2 + b2) * ts.n1 + e1 + b1]
                                if fa >= 0 and fb >= 0:
                                    ref[fa, fb] += np.sum(wt * B1[:, a1] * B2[:, a2] * B1[:, b1] * B2[:, b2])
    np.testing.assert_allclose(G, ref, rtol=0, atol=1e-15)


def test_circle_entries_bruteforce():
    """A few cut-row entries (c = 1) by adaptive quadrature with exact inner integrals."""
    cfg = wl.config1(N=8)
    o = _const(cfg)
    G = o.gauss_reference().tocsr()
    ts = o.ts
    p, k1, k2 = ts.p, ts.knots1, ts.knots2
    gy, wy = np.polynomial.legendre.leggauss(p + 2)
    rng = np.random.default_rng(0)
    cut_rows = np.nonzero(ts.fcls.reshape(-1) == 2)[0]
    for f in rng.choice(cut_rows, 6, replace=False):
        i2, i1 = divmod(int(f), ts.n1)
        r = ts.act_of[f]
        row = G.getrow(r)
        for c, v in zip(row.indices[:5], row.data[:5]):
            j2, j1 = divmod(int(ts.active[c]), ts.n1)

            def inner(x):
                # visible y-intervals at abscissa x, then Gauss on each element piece
                dx = x - 0.5
                holes = []
                if abs(dx) < 0.25:
                    h = math.sqrt(0.0625 - dx * dx)
                    holes = [(0.5 - h, 0.5 + h)]
                e1 = int(bspline.element_of(ts.bp1, x))
                bx = bspline.basis(k1, p, i1, np.array([x]), e1)[0] * bspline.basis(k1, p, j1, np.array([x]), e1)[0]
                if bx == 0.0:
                    return 0.0
                tot = 0.0
                for e2 in range(ts.N2):
                    ya, yb = ts.bp2[e2], ts.bp2[e2 + 1]
                    pieces = [(ya, yb)]
                    for (ha, hb) in holes:
                        new = []
                        for (a, b) in pieces:
                            if hb <= a or ha >= b:
                                new.append((a, b))
                            else:
                                if a < ha:
                                    new.append((a, ha))
                                if hb < b:
                                    new.append((hb, b))
                        pieces = new
                    for (a, b) in pieces:
                        yy = a + (b - a) * (gy + 1) / 2
                        B = bspline.basis(k2, p, i2, yy, e2) * bspline.basis(k2, p, j2, yy, e2)
                        tot += np.sum(wy * (b - a) / 2 * B)
                return bx * tot

            pts = sorted(set(list(ts.bp1[1:-1]) + [0.25, 0.75]))
            ref, _ = integrate.quad(inner, 0, 1, points=pts, limit=400, epsabs=1e-15, epsrel=1e-12)
            assert abs(v - ref) < 1e-11 * max(abs(ref), 1e-5)


def test_detj_total_is_mapped_area():
    """Untrimmed, c = |det J| with det J > 0: sum of M = area of the mapped square.

    The area comes from Green's theorem on the four mapped edges, each a
    B-spline curve of the patch's own degree evaluated by SciPy.
    """
    from scipy.interpolate import BSpline
    cfg = wl.config2(N=10, p=3)
    cfg.curves = []
    o = Oracle(cfg)
    P = cfg.geom_cp
    k1, k2 = o.ts.knots1, o.ts.knots2
    p = cfg.p
    # det J > 0 on a fine sample, so |det J| = det J
    xs = np.linspace(0, 1, 41)
    _, _, D = map_and_detj(cfg, np.repeat(xs, 41), np.tile(xs, 41))
    assert D.min() > 0
    edges = [(k1, P[0, :, :], 1.0), (k2, P[:, -1, :], 1.0), (k1, P[-1, :, :], -1.0), (k2, P[:, 0, :], -1.0)]
    g, w = np.polynomial.legendre.leggauss(2 * p + 2)
    area = 0.0
    for knots, cp, sgn in edges:
        sx, sy = BSpline(knots, cp[:, 0], p), BSpline(knots, cp[:, 1], p)
        dsy = sy.derivative()
        bp = np.unique(knots)
        for a, b in zip(bp[:-1], bp[1:]):
            t = a + (b - a) * (g + 1) / 2
            area += sgn * np.sum(w * (b - a) / 2 * sx(t) * dsy(t))
    assert abs(o.gauss_reference().sum() - area) < 1e-13


def test_ell_roundtrip():
    o = _const(wl.config1(N=10))
    H = o.hybrid()
    assert abs(from_ell(to_ell(H, o.ts), o.ts) - H).max() == 0.0
