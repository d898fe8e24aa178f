"""B-splines (Sect. 2.1) written as their defining recursion.

A B-spline B_{i,p} over knot vector Xi is piecewise polynomial of degree p,
supported on [xi_i, xi_{i+p+1}]; each non-empty knot span is an element and
carries p+1 non-zero B-splines. The bivariate basis is the tensor product of
Eq. (1). The recursion itself (Cox-de Boor) is the textbook definition; the
paper states only its properties.

Reading: points are always evaluated *element-locally* -- the caller names the
element that owns the point, so the half-open convention at knots never
matters (degree-0 functions are 1 on the named element's span).
"""
from __future__ import annotations

import numpy as np


def breakpoints(knots, p):
    """Distinct knot values; element e is [bp[e], bp[e+1]].

    Only open knot vectors with simple interior knots (maximal smoothness
    C^{p-1}) are handled, which is the setting of every experiment here.
    """
    knots = np.asarray(knots, dtype=np.float64)
    bp = np.unique(knots)
    assert np.all(knots[:p + 1] == knots[0]) and np.all(knots[-p - 1:] == knots[-1])
    assert len(knots) == len(bp) + 2 * p, "interior knots must be simple"
    return bp


def n_functions(knots, p):
    return len(knots) - p - 1


def _degree_table(knots, p, x, span):
    """Values B_{j,r}(x) for r = 0..p, built bottom-up from the recursion.

    B_{j,0} = [j == span]; B_{j,r} = (x - xi_j)/(xi_{j+r} - xi_j) B_{j,r-1}
    + (xi_{j+r+1} - x)/(xi_{j+r+1} - xi_{j+1}) B_{j+1,r-1} (0/0 terms dropped).
    Returns a list over r of dicts j -> values.
    """
    table = [{span: np.ones_like(x)}]
    for r in range(1, p + 1):
        prev, cur = table[-1], {}
        for j in range(span - r, span + 1):
            v = np.zeros_like(x)
            d1 = knots[j + r] - knots[j]
            if d1 > 0 and j in prev:
                v = v + (x - knots[j]) / d1 * prev[j]
            d2 = knots[j + r + 1] - knots[j + 1]
            if d2 > 0 and (j + 1) in prev:
                v = v + (knots[j + r + 1] - x) / d2 * prev[j + 1]
            cur[j] = v
        table.append(cur)
    return table


def _basis_recursive(knots, p, i, x, span):
    """B_{i,p}(x) by the recursion, with B_{i,0} = [i == span]."""
    return _degree_table(knots, p, x, span)[p].get(i, np.zeros_like(x))


def basis(knots, p, i, x, e):
    """Value of B_{i,p} at points x that all lie in element e."""
    x = np.asarray(x, dtype=np.float64)
    span = p + e
    return _basis_recursive(np.asarray(knots, dtype=np.float64), p, i, x, span)


def basis_deriv(knots, p, i, x, e):
    """Derivative of B_{i,p}: p/(xi_{i+p}-xi_i) B_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) B_{i+1,p-1}."""
    knots = np.asarray(knots, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    span = p + e
    out = np.zeros_like(x)
    if p == 0:
        return out
    d1 = knots[i + p] - knots[i]
    if d1 > 0:
        out += p / d1 * _basis_recursive(knots, p - 1, i, x, span)
    d2 = knots[i + p + 1] - knots[i + 1]
    if d2 > 0:
        out -= p / d2 * _basis_recursive(knots, p - 1, i + 1, x, span)
    return out


def local_basis(knots, p, e, x):
    """(len(x), p+1) array of B_{e..e+p} at points x in element e."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    tab = _degree_table(np.asarray(knots, dtype=np.float64), p, x, p + e)[p]
    return np.stack([tab[e + a] for a in range(p + 1)], axis=1)


def local_basis_deriv(knots, p, e, x):
    """(len(x), p+1) derivatives of B_{e..e+p} at points x in element e."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if p == 0:
        return np.zeros((x.size, 1))
    knots = np.asarray(knots, dtype=np.float64)
    low = _degree_table(knots, p, x, p + e)[p - 1]
    cols = []
    for a in range(p + 1):
        i = e + a
        v = np.zeros_like(x)
        d1 = knots[i + p] - knots[i]
        if d1 > 0 and i in low:
            v = v + p / d1 * low[i]
        d2 = knots[i + p + 1] - knots[i + 1]
        if d2 > 0 and (i + 1) in low:
            v = v - p / d2 * low[i + 1]
        cols.append(v)
    return np.stack(cols, axis=1)


def element_of(bp, x):
    """Element containing x (last element for x == end)."""
    e = np.searchsorted(bp, x, side="right") - 1
    return np.clip(e, 0, len(bp) - 2)


def support_elements(p, n_el, i):
    """Elements e with B_i non-zero on e: e in [i-p, i] within [0, n_el)."""
    return range(max(0, i - p), min(n_el - 1, i) + 1)
