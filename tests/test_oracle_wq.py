"""Pins of the oracle's weighted quadrature (Eqs. (4)-(5)) on the CPU."""
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from oracle import bspline, wq
from oracle.assemble import Oracle
from oracle.geometry import Coefficient
from paper_2101_08053_amd import workloads as wl


def _exact_mass_uniform(N, p):
    """Exact univariate mass matrix on open uniform knots, by symbolic integration."""
    t = sp.symbols("t")
    knots = [sp.Integer(0)] * p + [sp.Rational(k, N) for k in range(N + 1)] + [sp.Integer(1)] * p
    n = N + p

    def piece(i, r, e):
        # B_{i,r} on element e as a sympy expression, via the recursion
        if r == 0:
            return sp.Integer(1) if i == p + e else sp.Integer(0)
        out = sp.Integer(0)
        d1 = knots[i + r] - knots[i]
        if d1 != 0:
            out += (t - knots[i]) / d1 * piece(i, r - 1, e)
        d2 = knots[i + r + 1] - knots[i + 1]
        if d2 != 0:
            out += (knots[i + r + 1] - t) / d2 * piece(i + 1, r - 1, e)
        return sp.expand(out)

    M = [[Fraction(0)] * n for _ in range(n)]
    for e in range(N):
        loc = [piece(e + a, p, e) for a in range(p + 1)]
        a0, b0 = sp.Rational(e, N), sp.Rational(e + 1, N)
        for a in range(p + 1):
            for b in range(p + 1):
                v = sp.integrate(loc[a] * loc[b], (t, a0, b0))
                M[e + a][e + b] += Fraction(int(v.p), int(v.q))
    return M


@pytest.mark.parametrize("N,p", [(4, 1), (5, 2), (6, 3)])
def test_mass_1d_exact_rationals(N, p):
    M = wq.mass_1d(wl.open_uniform_knots(N, p), p)
    ex = _exact_mass_uniform(N, p)
    ref = np.array([[float(v) for v in row] for row in ex])
    np.testing.assert_allclose(M, ref, rtol=0, atol=1e-16)


@pytest.mark.parametrize("N,p", [(3, 1), (10, 2), (12, 4), (9, 6), (1, 3), (2, 5)])
def test_wq_layout(N, p):
    knots = wl.open_uniform_knots(N, p)
    xs, el = wq.wq_points(knots, p)
    bp = bspline.breakpoints(knots, p)
    assert len(xs) == (2 * N + 2 * p - 2 if N >= 2 else p + 1)
    # no point on a knot, each point inside its element
    assert np.all(xs > bp[el]) and np.all(xs < bp[el + 1])
    assert np.min(np.abs(xs[:, None] - bp[None, :])) > 0


@pytest.mark.parametrize("N,p", [(10, 1), (10, 2), (12, 4), (9, 6), (2, 3), (16, 5)])
def test_wq_exactness_eq5(N, p):
    knots = wl.open_uniform_knots(N, p)
    W, res = wq.wq_weights(knots, p, return_residual=True)
    assert res < 1e-14
    # weights vanish outside the support of the test function
    xs, el = wq.wq_points(knots, p)
    for i in range(W.shape[0]):
        outside = (el < i - p) | (el > i)
        assert np.all(W[i, outside] == 0.0)


def test_wq_exactness_nonuniform():
    k = np.concatenate([np.zeros(4), [0.1, 0.15, 0.4, 0.72, 0.9], np.ones(4)])
    W, res = wq.wq_weights(k, 3, return_residual=True)
    assert res < 1e-14


@pytest.mark.parametrize("N1,N2,p", [(6, 5, 2), (5, 7, 3), (8, 8, 4)])
def test_untrimmed_wq_is_kronecker(N1, N2, p):
    """Untrimmed, c = 1: the WQ matrix equals M2 (x) M1 with i = i2 n1 + i1."""
    patch = wl.Patch(p=p, n_el=(N1, N2), knots=(wl.open_uniform_knots(N1, p), wl.open_uniform_knots(N2, p)),
                     curves=[], coef=wl.COEF_CONST)
    o = Oracle(patch, coef=Coefficient(patch, kind=wl.COEF_CONST))
    M = o.wq_rows(o.ts.active).toarray()
    K = np.kron(wq.mass_1d(patch.knots[1], p), wq.mass_1d(patch.knots[0], p))
    np.testing.assert_allclose(M, K, rtol=0, atol=1e-13 * np.abs(K).max())
