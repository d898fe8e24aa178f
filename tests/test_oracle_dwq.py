"""Pins of the oracle's discontinuous weighted quadrature (Sect. 3.3, Eqs. (9)-(10)).

* knot insertion: the subdivision matrix against SciPy's knot insertion and
  against direct evaluation of the refined basis;
* nested points (largest resulting gap first) against their closed form;
* the 1-D rule's defining property (separability at t): on each side of t
  it integrates B_j B_i exactly for every trial function j;
* the box choice (largest inside box, fewer discontinuities, enumeration order) on hand-made class patterns;
* the 2-D DWQ matrix against element-wise Gauss at c = 1 (Table 1, middle
  column) and its area invariant.
"""
import json
import os

import numpy as np
import pytest
from scipy import interpolate

from oracle import bspline, dwq
from oracle.assemble import Oracle
from oracle.geometry import Coefficient
from oracle.quadrature import gauss_on
from paper_2101_08053_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_massmatrix_error.json")


def _open_knots(p, N, rng=None):
    inner = np.arange(1, N) / N
    if rng is not None:   # non-uniform simple interior knots
        inner = np.sort(inner + rng.uniform(-0.3, 0.3, N - 1) / N)
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_insertion_matrix_matches_scipy(p):
    rng = np.random.default_rng(p)
    kv = _open_knots(p, 7, rng)
    n = len(kv) - p - 1
    t = kv[p + 3]            # an existing simple interior knot
    kr, S = dwq.insert_knot(kv, p, t, p)
    assert np.sum(kr == t) == p + 1
    P = rng.standard_normal(n)
    tck = (kv, P, p)
    for _ in range(p):
        tck = interpolate.insert(t, tck, m=1)
    np.testing.assert_allclose(S @ P, tck[1][:len(kr) - p - 1], rtol=0, atol=1e-13)
    # B_j = sum_l S[l, j] B~_l at random points (SciPy's evaluation of both bases)
    x = rng.uniform(0, 1, 50)
    for j in range(n):
        cj = np.zeros(n)
        cj[j] = 1.0
        lhs = interpolate.BSpline(kv, cj, p)(x)
        rhs = interpolate.BSpline(kr, S[:, j], p)(x)
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_nested_points_closed_form(p):
    a, b = 0.25, 0.375
    h = b - a
    existing = [a + h / 3, a + 2 * h / 3]
    for t, order in ((a, [0, 1, 2]), (b, [2, 1, 0])):
        got = dwq.nested_points(a, b, existing, p - 1, t)
        cnt = [0, 0, 0]
        for k in range(p - 1):      # equal gaps: round robin starting next to t
            cnt[order[k % 3]] += 1
        ref = sorted(a + h * (g + k / (cnt[g] + 1)) / 3 for g in range(3) for k in range(1, cnt[g] + 1))
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)
        allp = np.concatenate([got, existing])
        assert len(np.unique(allp)) == p + 1 and np.all((allp > a) & (allp < b))


def _side_integral(kv, p, i, j, t, side):
    """int over the side of t of B_i B_j, element Gauss with p+1 points (exact)."""
    bp = bspline.breakpoints(kv, p)
    tot = 0.0
    for e in range(len(bp) - 1):
        if (side == dwq.HIGH and bp[e] < t) or (side == dwq.LOW and bp[e + 1] > t):
            continue
        x, w = gauss_on(p + 1, bp[e], bp[e + 1])
        B = bspline.local_basis(kv, p, e, x)
        if e <= i <= e + p and e <= j <= e + p:
            tot += np.sum(w * B[:, i - e] * B[:, j - e])
    return tot


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("uniform", [True, False])
def test_dwq_rule_is_separable(p, uniform):
    """sum_{k on the side} w^_{k,i} B_j(x_k) = int_side B_j B_i for every j (the rule's purpose)."""
    kv = _open_knots(p, 9, None if uniform else np.random.default_rng(10 + p))
    D = dwq.Direction(kv, p)
    worst = 0.0
    for s in range(1, D.N):
        t = D.bp[s]
        for side in (dwq.LOW, dwq.HIGH):
            for i in range(s, s + p):
                x, el, _, w = D.dwq_weights(i, s, side)
                assert np.all(x > t) if side == dwq.HIGH else np.all(x < t)
                for j in range(max(0, i - p), min(D.n - 1, i + p) + 1):
                    Bj = np.array([bspline.local_basis(kv, p, e, [xx])[0, j - e] if e <= j <= e + p else 0.0
                                   for xx, e in zip(x, el)])
                    ref = _side_integral(kv, p, i, j, t, side)
                    worst = max(worst, abs(w @ Bj - ref) / D.bp[-1])
    assert worst <= 1e-14


def test_dwq_rule_reduces_to_coarse_far_from_t():
    """Points of the side not in supp B_i carry zero weight."""
    p = 3
    D = dwq.Direction(_open_knots(p, 10), p)
    s = 4
    for i in range(s, s + p):
        x, el, _, w = D.dwq_weights(i, s, dwq.HIGH)
        assert np.all(w[el > i] == 0.0)
        x, el, _, w = D.dwq_weights(i, s, dwq.LOW)
        assert np.all(w[el < i - p] == 0.0)


def test_region_choice_patterns():
    p, N = 2, 8
    i1 = i2 = 4                  # support elements 2..4 in both directions
    base = np.ones((N, N), dtype=bool)
    # cut corner at the low end of both directions: whole x range, above knot 3
    ins = base.copy()
    ins[2, 2] = False
    assert dwq.choose_region(ins, i1, i2, p, N, N) == ((2, 4, -1, -1), (3, 4, 3, dwq.HIGH))
    # centre element cut: a 3x1 strip, the first one met is the top row (high side)
    ins = base.copy()
    ins[3, 3] = False
    assert dwq.choose_region(ins, i1, i2, p, N, N) == ((2, 4, -1, -1), (4, 4, 4, dwq.HIGH))
    # whole left column cut: direction 1 above knot 3, direction 2 whole
    ins = base.copy()
    ins[2:5, 2] = False
    assert dwq.choose_region(ins, i1, i2, p, N, N) == ((3, 4, 3, dwq.HIGH), (2, 4, -1, -1))
    # top-right corner cut: whole x below knot 4 (3 elements x 2) ties with the
    # column pair (2 x 3); direction-1 options are outer, so (whole, low) wins
    ins = base.copy()
    ins[4, 4] = False
    assert dwq.choose_region(ins, i1, i2, p, N, N) == ((2, 4, -1, -1), (2, 3, 4, dwq.LOW))
    # nothing inside
    ins = np.zeros((N, N), dtype=bool)
    assert dwq.choose_region(ins, i1, i2, p, N, N) is None


def _const(cfg):
    return Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_CONST))


def test_table1_dwq_column():
    """DWQ agrees with element Gauss at round-off (Table 1, middle column)."""
    gold = json.load(open(GOLDEN))["rows"]
    for p in range(1, 7):
        o = _const(wl.table1_line(p))
        G = o.gauss_reference().toarray()
        e = np.linalg.norm(o.dwq().toarray() - G)
        assert e <= max(gold[str(p)][1], 1e-16) * 10


@pytest.mark.parametrize("cfg", [wl.config1(N=16), wl.config2(N=12, p=4), wl.config3(N=12, p=3),
                                 wl.nonuniform_variant(wl.config1(N=16, p=3))],
                         ids=lambda c: c.name)
def test_dwq_equals_gauss_at_c1(cfg):
    o = _const(cfg)
    G = o.gauss_reference()
    D = o.dwq()
    scale = np.abs(G).max()
    assert np.abs((D - G).toarray()).max() <= 1e-13 * scale
    assert abs(D.sum() - o.ts.visible_area()) <= 1e-13
    # some rows really use a box with a discontinuity in each case
    regs = [o.dwq_region(*divmod(int(f), o.ts.n1)[::-1]) for f in o.cut_rows_flat()]
    assert sum(r is not None and (r[0][2] >= 0 or r[1][2] >= 0) for r in regs) > 0
