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


def _separable_patch(p=3, N=10):
    """Line-trimmed patch with a separable map F(x, y) = (f(x), g(y)): c = |det J| = f'(x) g'(y)."""
    cfg = wl.table1_line(p, N=N)
    g1 = wl.greville(cfg.knots[0], p)
    g2 = wl.greville(cfg.knots[1], p)
    a = g1 + 0.2 * g1 ** 2            # increasing: f' > 0
    b = g2 - 0.15 * g2 ** 2           # increasing: g' > 0
    cp = np.empty((len(g2), len(g1), 2))
    cp[..., 0] = a[None, :]
    cp[..., 1] = b[:, None]
    cfg.geom_cp = cp
    cfg.coef = wl.COEF_GEOM_DETJ
    return cfg, a, b


def _factor_1d(knots, p, coefs, x, w):
    """sum_k w_k f'(x_k) B_j(x_k) for every j, f = sum_i coefs_i B_i (SciPy evaluation)."""
    from scipy.interpolate import BSpline
    fp = BSpline(knots, coefs, p).derivative()(x)
    B = BSpline.design_matrix(x, knots, p).toarray()
    return (w * fp) @ B


def test_wq_rows_separable_coefficient():
    """WQ interior rows with a non-constant c pinned by separability (Eqs. (5)-(7)).

    For c(x, y) = c1(x) c2(y) the double sum of Eq. (7) factorises: the entry
    (i, j) is (sum_k w1_{k,i1} c1 B_j1)(sum_l w2_{l,i2} c2 B_j2). Here c is
    |det J| of a separable map, whose factors f', g' and the basis values are
    evaluated by SciPy; the oracle's rows come from its two-dimensional grid of
    c and its tensor sums. c is not symmetric in (i, j), so an exchanged test
    and trial index fails as well as a wrong direction or a wrong c.
    """
    cfg, a, b = _separable_patch()
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_GEOM_DETJ))
    p, n1 = cfg.p, o.ts.n1
    k1, k2 = o.k1, o.k2
    rows = o.interior_rows_flat()
    assert len(rows) > 20
    worst = 0.0
    for f in rows:
        i2, i1 = divmod(int(f), n1)
        F1 = _factor_1d(k1, p, a, o.xs1, o.W1[i1])
        F2 = _factor_1d(k2, p, b, o.xs2, o.W2[i2])
        row = o.wq_row(i1, i2)
        scale = max(abs(v) for v in row.values())
        for col, v in row.items():
            j2, j1 = divmod(col, n1)
            worst = max(worst, abs(v - F1[j1] * F2[j2]) / scale)
    assert worst < 1e-13, worst
    # the coefficient is far from constant, so the pin is not the c = 1 case
    c = o.wq_grid_coef()
    assert c.max() / c.min() > 1.3


def test_dwq_box_separable_coefficient():
    """DWQ rows (Sect. 3.3) with a non-constant c: the box part factorises like a WQ row.

    Each DWQ row is its box's tensor rule plus element rules on the rest of
    its support. With c = f'(x) g'(y) the box part is the product of the two
    1-D refined sums (SciPy values of f', g' and the basis), so the row minus
    its element-rule part must equal that product.
    """
    cfg, a, b = _separable_patch()
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_GEOM_DETJ))
    p, ts = cfg.p, o.ts
    n1 = ts.n1
    from oracle.trim import CUT, INSIDE
    checked = 0
    worst = 0.0
    for f in o.cut_rows_flat():
        i2, i1 = divmod(int(f), n1)
        reg = o.dwq_region(i1, i2)
        if reg is None:
            continue
        o1, o2 = reg
        x1, _, _, w1 = o.dwq_rule(0, i1, o1)
        x2, _, _, w2 = o.dwq_rule(1, i2, o2)
        F1 = _factor_1d(o.k1, p, a, x1, w1)
        F2 = _factor_1d(o.k2, p, b, x2, w2)
        row = dict(o.dwq_row(i1, i2))
        for e2 in range(max(0, i2 - p), min(ts.N2 - 1, i2) + 1):   # take away the element-rule part
            for e1 in range(max(0, i1 - p), min(ts.N1 - 1, i1) + 1):
                if (o1[0] <= e1 <= o1[1] and o2[0] <= e2 <= o2[1]) or ts.ecls[e2, e1] not in (INSIDE, CUT):
                    continue
                E = o.local_matrix(e1, e2)
                li = (i2 - e2) * (p + 1) + (i1 - e1)
                for a2 in range(p + 1):
                    for a1 in range(p + 1):
                        col = (e2 + a2) * n1 + (e1 + a1)
                        row[col] -= E[li, a2 * (p + 1) + a1]
        scale = max(abs(v) for v in row.values())
        for col, v in row.items():
            j2, j1 = divmod(col, n1)
            worst = max(worst, abs(v - F1[j1] * F2[j2]) / scale)
        checked += 1
    assert checked >= 5
    assert worst < 1e-12, worst
