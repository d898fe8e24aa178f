"""Weighted quadrature in one direction (Sect. 2.1, Eqs. (4)-(5)).

One rule Q_i per test function B_i: points x_k, weights w_{k,i} with
    sum_k B_j(x_k) w_{k,i} = int B_j B_i  for every trial B_j overlapping B_i,
over the points k that lie in supp B_i; weights outside supp B_i are zero.

Readings (the point placement of the cited work is not in the paper):
* R1 point count: p+1 points in the first and last element, 2 in every other
  element (maximal smoothness, simple interior knots).
* R2 positions: uniform inside each element, a + (b-a) k/(n_e+1), k = 1..n_e,
  so no point lies on a knot.
* R3 solution of the under-determined system (5): the minimum 2-norm solution.
  The oracle takes NumPy's least-squares routine (SVD based) for it.
"""
from __future__ import annotations

import numpy as np

from . import bspline
from .quadrature import gauss_on


def points_per_element(n_el, p):
    return np.array([p + 1 if (e == 0 or e == n_el - 1) else 2 for e in range(n_el)], dtype=np.int64)


def wq_points(knots, p):
    """Point coordinates and owning element of the one-direction WQ layout (R1, R2)."""
    bp = bspline.breakpoints(knots, p)
    n_el = len(bp) - 1
    xs, el = [], []
    for e, ne in enumerate(points_per_element(n_el, p)):
        a, b = bp[e], bp[e + 1]
        for k in range(1, ne + 1):
            xs.append(a + (b - a) * k / (ne + 1))
            el.append(e)
    return np.array(xs), np.array(el, dtype=np.int64)


def mass_1d(knots, p):
    """Exact univariate mass matrix int B_i B_j by (p+1)-point Gauss per element."""
    bp = bspline.breakpoints(knots, p)
    n = bspline.n_functions(knots, p)
    M = np.zeros((n, n))
    for e in range(len(bp) - 1):
        x, w = gauss_on(p + 1, bp[e], bp[e + 1])
        B = bspline.local_basis(knots, p, e, x)
        M[e:e + p + 1, e:e + p + 1] += np.einsum("g,ga,gb->ab", w, B, B)
    return M


def basis_at_points(knots, p, xs, el):
    """Dense (len(xs), n) table B_j(x_k), element-local."""
    n = bspline.n_functions(knots, p)
    T = np.zeros((len(xs), n))
    for e in np.unique(el):
        idx = np.nonzero(el == e)[0]
        T[np.ix_(idx, np.arange(e, e + p + 1))] = bspline.local_basis(knots, p, e, xs[idx])
    return T


def basis_deriv_at_points(knots, p, xs, el):
    """Dense (len(xs), n) table B_j'(x_k), element-local."""
    n = bspline.n_functions(knots, p)
    T = np.zeros((len(xs), n))
    for e in np.unique(el):
        idx = np.nonzero(el == e)[0]
        T[np.ix_(idx, np.arange(e, e + p + 1))] = bspline.local_basis_deriv(knots, p, e, xs[idx])
    return T


def wq_weights(knots, p, xs=None, el=None, M1=None, return_residual=False):
    """Dense (n, Q) weights W[i, k] = w_{k,i} solving Eq. (5) for every test function i."""
    if xs is None:
        xs, el = wq_points(knots, p)
    if M1 is None:
        M1 = mass_1d(knots, p)
    n_el = len(bspline.breakpoints(knots, p)) - 1
    n = bspline.n_functions(knots, p)
    T = basis_at_points(knots, p, xs, el)
    W = np.zeros((n, len(xs)))
    worst = 0.0
    for i in range(n):
        sup = list(bspline.support_elements(p, n_el, i))
        Qi = np.nonzero((el >= sup[0]) & (el <= sup[-1]))[0]
        Ji = np.arange(max(0, i - p), min(n - 1, i + p) + 1)
        A = T[np.ix_(Qi, Ji)].T
        b = M1[Ji, i]
        w = np.linalg.lstsq(A, b, rcond=None)[0]
        W[i, Qi] = w
        worst = max(worst, np.linalg.norm(A @ w - b) / np.linalg.norm(b))
    if return_residual:
        return W, worst
    return W


def wq_condition(knots, p, xs=None, el=None):
    """2-norm condition number of each system (5) (NumPy's routine), per test function."""
    if xs is None:
        xs, el = wq_points(knots, p)
    n_el = len(bspline.breakpoints(knots, p)) - 1
    n = bspline.n_functions(knots, p)
    T = basis_at_points(knots, p, xs, el)
    out = np.zeros(n)
    for i in range(n):
        sup = list(bspline.support_elements(p, n_el, i))
        Qi = np.nonzero((el >= sup[0]) & (el <= sup[-1]))[0]
        Ji = np.arange(max(0, i - p), min(n - 1, i + p) + 1)
        out[i] = np.linalg.cond(T[np.ix_(Qi, Ji)].T)
    return out
