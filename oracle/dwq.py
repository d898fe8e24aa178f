"""Discontinuous weighted quadrature (Sect. 3.3, Eqs. (9)-(10)).

Test infrastructure: plain and slow, written from the paper's construction
for checking the device path; nothing here is used by the library.

For a test function B_i whose support contains an interior knot t, a rule on
one side of t (the "high" side x > t or the "low" side x < t) is built so
that, for every trial function B_j,

    sum_{k on the side} w^_{k,i} B_j(x_k) = int_{side} B_j B_i .

Steps, in the paper's order:
 1. insert t until it has multiplicity p+1 (the refined basis is C^-1 at t);
    the subdivision matrix S of Eq. (10) relates the bases by
    B_i = sum_l S[l, i] B~_l (reading R7: this is the function relation that
    follows from the control-point relation (9) by linearity);
 2. the element next to t on the chosen side gets p+1 points (reading R10:
    like an end element); the missing points are nested between the existing
    ones (reading R9, the remark after the construction);
 3. the weighted-quadrature system (5) of the refined space is solved, in
    minimum norm, for every refined function l on the side with
    S[l, i] != 0 (these are the functions touching the element next to t);
 4. w^_{k,i} = sum_l S[l, i] w~_{k,l}.

The 2-D use (Sect. 3.3, last part; reading R8): for a cut function i the
region R of its support that is integrated by sum factorisation is a box
I1 x I2 of inside elements, each I_d being the whole support range, or the
part of it above or below one interior knot. The rest of the support is
integrated element by element (Gauss on inside elements, the cut rule on cut
elements).
"""
from __future__ import annotations

import numpy as np

from . import bspline, wq
from .quadrature import gauss_on

LOW, HIGH = 0, 1


# ------------------------------------------------------------ Eq. (10)
def insert_knot(knots, p, t, times=1):
    """Refined knot vector and S (n_refined x n) with B_j = sum_l S[l, j] B~_l.

    One insertion of t in [u_s, u_{s+1}) maps coefficients by
    S(c, c-1) = 1 - alpha_c, S(c, c) = alpha_c with alpha_c = 1 for
    c <= s - p, (t - u_c)/(u_{c+p} - u_c) for s-p+1 <= c <= s, 0 otherwise
    (Eq. (10)); repeated insertions multiply the single-knot matrices.
    """
    kv = np.asarray(knots, dtype=np.float64).copy()
    n = len(kv) - p - 1
    S = np.eye(n)
    for _ in range(times):
        s = int(np.searchsorted(kv, t, side="right")) - 1
        m = len(kv) - p - 1
        S1 = np.zeros((m + 1, m))
        for c in range(m + 1):
            if c <= s - p:
                alpha = 1.0
            elif c <= s:
                alpha = (t - kv[c]) / (kv[c + p] - kv[c])
            else:
                alpha = 0.0
            if c < m:
                S1[c, c] = alpha
            if c >= 1:
                S1[c, c - 1] = 1.0 - alpha
        S = S1 @ S
        kv = np.insert(kv, s + 1, t)
    return kv, S


def span_basis(knots, p, span, x):
    """(len(x), p+1) values of B_{span-p..span} at x in [u_span, u_span+1] (Cox-de Boor)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    tab = bspline._degree_table(np.asarray(knots, dtype=np.float64), p, x, span)[p]
    return np.stack([tab[span - p + a] for a in range(p + 1)], axis=1)


# -------------------------------------------------------------- R9 points
def nested_points(a, b, existing, n_add, t):
    """Points added inside [a, b] between the existing ones (reading R9).

    The gaps are the intervals between consecutive existing points, with a and
    b as outer ends. Points are added one at a time to the gap whose spacing
    after the addition is largest; ties go to the gap nearest t, then to the
    lower one. Inside a gap the points are equispaced.
    """
    ends = [a] + sorted(existing) + [b]
    gaps = [(ends[g], ends[g + 1]) for g in range(len(ends) - 1)]
    cnt = [0] * len(gaps)
    h = b - a
    for _ in range(n_add):
        best = None
        for g, (lo, hi) in enumerate(gaps):
            spacing = (hi - lo) / (cnt[g] + 2)
            dist = min(abs(lo - t), abs(hi - t))
            key = (spacing, -dist, -lo)
            if best is None or _better(key, best[0], h):
                best = (key, g)
        cnt[best[1]] += 1
    out = []
    for g, (lo, hi) in enumerate(gaps):
        for k in range(1, cnt[g] + 1):
            out.append(lo + (hi - lo) * k / (cnt[g] + 1))
    return np.array(sorted(out))


def _better(key, best, h):
    tol = 1e-12 * h
    if key[0] > best[0] + tol:
        return True
    if key[0] < best[0] - tol:
        return False
    if key[1] > best[1] + tol:
        return True
    if key[1] < best[1] - tol:
        return False
    return key[2] > best[2]


# ------------------------------------------------------------ 1-D rule
class Direction:
    """One parametric direction: knots, WQ points, coarse weights."""

    def __init__(self, knots, p):
        self.knots = np.asarray(knots, dtype=np.float64)
        self.p = p
        self.bp = bspline.breakpoints(self.knots, p)
        self.N = len(self.bp) - 1
        self.n = bspline.n_functions(self.knots, p)
        self.xs, self.el = wq.wq_points(self.knots, p)
        self.W = wq.wq_weights(self.knots, p, self.xs, self.el)
        self._cache = {}
        self._cond = {}

    def side_rule(self, s, side):
        """Refined points of the side of t = bp[s] and the weights w~ of its refined functions.

        Returns (x, el, kidx, S, l_side, Wt): points in increasing x with their
        element and coarse point index (-1 for nested points); S of Eq. (10);
        the refined functions l on the side that touch the element next to t;
        Wt[r] = weights of refined function l_side[r] on the points.
        """
        key = (s, side)
        if key in self._cache:
            return self._cache[key]
        p, bp = self.p, self.bp
        assert 1 <= s <= self.N - 1, "the discontinuity must be an interior knot"
        t = bp[s]
        kv, S = insert_knot(self.knots, p, t, p)   # t: multiplicity 1 -> p+1
        e_adj = s if side == HIGH else s - 1
        # refined point set on the side: coarse points plus nested ones in e_adj
        on_side = (self.el >= s) if side == HIGH else (self.el <= s - 1)
        kidx = list(np.nonzero(on_side)[0])
        x = list(self.xs[kidx])
        el = list(self.el[kidx])
        n_have = int(np.sum(self.el == e_adj))
        n_add = max(0, (p + 1) - n_have)
        if n_add:
            a, b = bp[e_adj], bp[e_adj + 1]
            add = nested_points(a, b, list(self.xs[self.el == e_adj]), n_add, t)
            x += list(add)
            el += [e_adj] * len(add)
            kidx += [-1] * len(add)
        order = np.argsort(np.asarray(x), kind="stable")
        x = np.asarray(x)[order]
        el = np.asarray(el)[order]
        kidx = np.asarray(kidx)[order]
        # refined functions on the side
        n_ref = len(kv) - p - 1
        if side == HIGH:
            side_fns = [l for l in range(n_ref) if kv[l] >= t]
        else:
            side_fns = [l for l in range(n_ref) if kv[l + p + 1] <= t]
        touch = [l for l in side_fns if kv[l] <= bp[e_adj] and kv[l + p + 1] >= bp[e_adj + 1]]
        # refined basis at the points: element e -> span = last knot index <= bp[e] in kv
        Tr = np.zeros((len(x), n_ref))
        for e in np.unique(el):
            idx = np.nonzero(el == e)[0]
            span = int(np.searchsorted(kv, bp[e], side="right")) - 1
            Tr[np.ix_(idx, np.arange(span - p, span + 1))] = span_basis(kv, p, span, x[idx])
        Wt = np.zeros((len(touch), len(x)))
        cond = 1.0
        for r, l in enumerate(touch):
            lo, hi = kv[l], kv[l + p + 1]
            Ql = np.nonzero((x > lo) & (x < hi))[0]
            Jl = [m for m in side_fns if abs(m - l) <= p]
            A = Tr[np.ix_(Ql, Jl)].T
            b = np.array([self._refined_moment(kv, m, l) for m in Jl])
            Wt[r, Ql] = np.linalg.lstsq(A, b, rcond=None)[0]
            cond = max(cond, float(np.linalg.cond(A)))
        out = (x, el, kidx, S, np.array(touch), Wt)
        self._cache[key] = out
        self._cond[key] = cond
        return out

    def side_condition(self, s, side):
        """Largest 2-norm condition number of the refined systems of the side of bp[s]."""
        self.side_rule(s, side)
        return self._cond[(s, side)]

    def _refined_moment(self, kv, m, l):
        """int B~_m B~_l, (p+1)-point Gauss on every element of the overlap."""
        p = self.p
        lo, hi = max(kv[m], kv[l]), min(kv[m + p + 1], kv[l + p + 1])
        tot = 0.0
        for e in range(self.N):
            a, b = self.bp[e], self.bp[e + 1]
            if a < lo or b > hi:
                continue
            span = int(np.searchsorted(kv, a, side="right")) - 1
            xg, wg = gauss_on(p + 1, a, b)
            B = span_basis(kv, p, span, xg)
            tot += np.sum(wg * B[:, m - (span - p)] * B[:, l - (span - p)])
        return tot

    def dwq_weights(self, i, s, side):
        """Points (x, el, kidx) of the side of bp[s] and the DWQ weights w^_{.,i} there."""
        x, el, kidx, S, touch, Wt = self.side_rule(s, side)
        w = np.zeros(len(x))
        for r, l in enumerate(touch):
            w += S[l, i] * Wt[r]
        return x, el, kidx, w

    def coarse_rule(self, i, elo, ehi):
        """Coarse WQ points of B_i inside elements [elo, ehi] and their weights."""
        k = np.nonzero((self.el >= elo) & (self.el <= ehi) & (self.W[i] != 0.0))[0]
        return self.xs[k], self.el[k], k, self.W[i, k]


# --------------------------------------------------------------- R8 region
def direction_options(lo, hi):
    """Ranges of one direction in preference order: whole; above knot s (s ascending); below s (s descending).

    Each option is (first element, last element, disc knot or -1, side or -1).
    """
    opts = [(lo, hi, -1, -1)]
    for s in range(lo + 1, hi + 1):
        opts.append((s, hi, s, HIGH))
    for s in range(hi, lo, -1):
        opts.append((lo, s - 1, s, LOW))
    return opts


def choose_region(inside, i1, i2, p, N1, N2):
    """Region R of the support of (i1, i2) integrated by DWQ (reading R8), or None.

    ``inside[e2, e1]`` is True for inside elements. Candidates pair one option
    per direction and must hold inside elements only. The largest one wins;
    ties go to fewer discontinuities, then to the first in the enumeration
    order (direction-1 options outer, direction-2 options inner).
    """
    lo1, hi1 = max(0, i1 - p), min(N1 - 1, i1)
    lo2, hi2 = max(0, i2 - p), min(N2 - 1, i2)
    best = None
    for o1 in direction_options(lo1, hi1):
        for o2 in direction_options(lo2, hi2):
            n_el = (o1[1] - o1[0] + 1) * (o2[1] - o2[0] + 1)
            if n_el <= 0 or not inside[o2[0]:o2[1] + 1, o1[0]:o1[1] + 1].all():
                continue
            nd = (o1[2] >= 0) + (o2[2] >= 0)
            if best is None or n_el > best[0] or (n_el == best[0] and nd < best[1]):
                best = (n_el, nd, o1, o2)
    if best is None:
        return None
    return best[2], best[3]
