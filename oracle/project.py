"""L2 projection on the trimmed patch (Sect. 4.2), written out plainly.

b_i is row i's own rule applied to g c (weighted quadrature for interior
rows, element Gauss and the cut rule for cut rows; with discontinuous
weighted quadrature, a cut row with a box R takes its box part from the
row's refined weights of Sect. 3.3 at the box's tensor points and the rest
of its support element by element, as its matrix row does); the system is solved with
A = (M + M^T)/2 (reading: the weighted-quadrature matrix is not symmetric when
c varies, so its symmetric part is used) by SciPy's direct sparse solver.
The relative L2 error uses a finer rule: (p+3)^2 Gauss points on inside
elements and the cut rule with two more inner and four more arc points.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import bspline
from .quadrature import gauss_on
from .trim import CUT, INSIDE


def _g_at(o, g, x, y, e1=None, e2=None):
    X, Y = o.coef.physical(x, y, e1, e2)
    return g(X, Y)


def rhs(o, g, method="hybrid", absolute=False):
    """b over active rows; ``g`` takes physical coordinates.

    ``absolute`` sums |w c g B_i| term by term instead: the scale of each
    entry's rounding error (B-splines are non-negative).
    """
    ab = np.abs if absolute else (lambda v: v)
    ts = o.ts
    b = np.zeros(ts.n_act)
    if method == "dwq":
        return _rhs_dwq(o, g, ab)
    if method == "hybrid":
        _rhs_wq_rows(o, g, ab, b)
        rows = o.cut_rows_flat()
        elements = o.cut_band_elements()
    else:
        rows = ts.active
        e2s, e1s = np.nonzero((ts.ecls == INSIDE) | (ts.ecls == CUT))
        elements = list(zip(e1s.tolist(), e2s.tolist()))
    keep = np.zeros(ts.n1 * ts.n2, dtype=bool)
    keep[np.asarray(rows, dtype=np.int64)] = True
    for (e1, e2) in elements:
        x, y, w = o.element_points(e1, e2)
        c = o.coef(x, y, e1, e2)
        gv = _g_at(o, g, x, y, e1, e2)
        B1 = bspline.local_basis(o.k1, o.p, e1, x)
        B2 = bspline.local_basis(o.k2, o.p, e2, y)
        for a2 in range(o.p + 1):
            for a1 in range(o.p + 1):
                f = (e2 + a2) * ts.n1 + e1 + a1
                if keep[f]:
                    b[ts.act_of[f]] += np.sum(ab(w * c * gv) * B1[:, a1] * B2[:, a2])
    return b


def _rhs_wq_rows(o, g, ab, b):
    """Interior rows: the row's weighted-quadrature weights on the WQ grid (Eq. (7) with B_j -> g)."""
    ts = o.ts
    cg = o.wq_grid_coef()
    X1 = np.repeat(o.xs1[:, None], len(o.xs2), axis=1)
    X2 = np.repeat(o.xs2[None, :], len(o.xs1), axis=0)
    E1 = np.repeat(o.el1[:, None], len(o.xs2), axis=1)
    E2 = np.repeat(o.el2[None, :], len(o.xs1), axis=0)
    G = _g_at(o, g, X1.ravel(), X2.ravel(), E1.ravel(), E2.ravel()).reshape(X1.shape) * cg
    for f in o.interior_rows_flat():
        i2, i1 = divmod(int(f), ts.n1)
        q1 = np.nonzero(o.W1[i1])[0]
        q2 = np.nonzero(o.W2[i2])[0]
        b[ts.act_of[f]] = np.einsum("k,l,kl->", ab(o.W1[i1, q1]), ab(o.W2[i2, q2]), ab(G[np.ix_(q1, q2)]))


def _element_vector(o, g, e1, e2, ab):
    """[a2, a1] -> sum over the element's rule of w c g B_(e1+a1) B_(e2+a2)."""
    x, y, w = o.element_points(e1, e2)
    t = ab(w * o.coef(x, y, e1, e2) * _g_at(o, g, x, y, e1, e2))
    B1 = bspline.local_basis(o.k1, o.p, e1, x)
    B2 = bspline.local_basis(o.k2, o.p, e2, y)
    return np.einsum("g,ga,gb->ba", t, ab(B1), ab(B2))


def _rhs_dwq(o, g, ab):
    """Discontinuous weighted quadrature (Sect. 3.3) with B_j -> g.

    A cut row with a box R (the box its matrix row uses): the row's 1-D rules restricted to R
    (the coarse WQ rule on a whole range, the refined weights of Eq. (10)
    otherwise) at their tensor points, plus the element rules of its inside
    and cut support elements outside R. A cut row without a box: element
    rules on its whole support.
    """
    ts, p = o.ts, o.p
    b = np.zeros(ts.n_act)
    _rhs_wq_rows(o, g, ab, b)
    cache = {}

    def vec(e1, e2):
        if (e1, e2) not in cache:
            cache[(e1, e2)] = _element_vector(o, g, e1, e2, ab)
        return cache[(e1, e2)]

    for f in o.cut_rows_flat():
        i2, i1 = divmod(int(f), ts.n1)
        reg = o.dwq_region(i1, i2)
        s = 0.0
        if reg is not None:
            o1, o2 = reg
            x1, el1, _, w1 = o.dwq_rule(0, i1, o1)
            x2, el2, _, w2 = o.dwq_rule(1, i2, o2)
            X = np.repeat(x1[:, None], len(x2), axis=1).ravel()
            Y = np.repeat(x2[None, :], len(x1), axis=0).ravel()
            E1 = np.repeat(el1[:, None], len(x2), axis=1).ravel()
            E2 = np.repeat(el2[None, :], len(x1), axis=0).ravel()
            GC = (o.coef(X, Y, E1, E2) * _g_at(o, g, X, Y, E1, E2)).reshape(len(x1), len(x2))
            s += np.einsum("k,l,kl->", ab(w1), ab(w2), ab(GC))
        for e2 in range(max(0, i2 - p), min(ts.N2 - 1, i2) + 1):
            for e1 in range(max(0, i1 - p), min(ts.N1 - 1, i1) + 1):
                if ts.ecls[e2, e1] not in (INSIDE, CUT):
                    continue
                if reg is not None and reg[0][0] <= e1 <= reg[0][1] and reg[1][0] <= e2 <= reg[1][1]:
                    continue
                s += vec(e1, e2)[i2 - e2, i1 - e1]
        b[ts.act_of[f]] = s
    return b


def solve(M, b):
    A = (0.5 * (M + M.T)).tocsc()
    return spla.spsolve(A, b)


def l2_error(o, u, g):
    """Relative L2(Omega_v, c) error of u_h = sum_active u_i B_i against g."""
    ts = o.ts
    p = o.p
    coeffs = np.zeros(ts.n1 * ts.n2)
    coeffs[ts.active] = u
    num = den = 0.0
    for e2 in range(ts.N2):
        for e1 in range(ts.N1):
            cls = ts.ecls[e2, e1]
            if cls == INSIDE:
                x1, w1 = gauss_on(p + 3, ts.bp1[e1], ts.bp1[e1 + 1])
                x2, w2 = gauss_on(p + 3, ts.bp2[e2], ts.bp2[e2 + 1])
                x = np.tile(x1, len(x2))
                y = np.repeat(x2, len(x1))
                w = np.outer(w2, w1).ravel()
            elif cls == CUT:
                x, y, w, _ = ts.cut_rule(e1, e2, n_r=ts.n_r + 2, n_s=ts.n_s + 2,
                                         n_q=max(ts.n_q(c) for c in ts.curves) + 4)
            else:
                continue
            c = o.coef(x, y, e1, e2)
            gv = _g_at(o, g, x, y, e1, e2)
            B1 = bspline.local_basis(o.k1, p, e1, x)
            B2 = bspline.local_basis(o.k2, p, e2, y)
            loc = coeffs[[(e2 + a2) * ts.n1 + e1 + a1 for a2 in range(p + 1) for a1 in range(p + 1)]]
            uh = np.einsum("ga,gb,ba->g", B1, B2, loc.reshape(p + 1, p + 1))
            num += np.sum(w * c * (uh - gv) ** 2)
            den += np.sum(w * c * gv ** 2)
    return np.sqrt(num / den)
