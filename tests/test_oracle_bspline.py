"""Pins of the oracle's B-spline layer against SciPy and closed forms (CPU)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline
from oracle.quadrature import gauss_on
from paper_2101_08053_amd import workloads as wl


def _knot_vectors():
    yield wl.open_uniform_knots(7, 1), 1
    yield wl.open_uniform_knots(9, 3), 3
    yield wl.open_uniform_knots(5, 6), 6
    # non-uniform simple interior knots
    k = np.concatenate([np.zeros(4), [0.1, 0.15, 0.4, 0.72, 0.9], np.ones(4)])
    yield k, 3


@pytest.mark.parametrize("kp", list(_knot_vectors()))
def test_basis_matches_scipy(kp):
    knots, p = kp
    bp = bspline.breakpoints(knots, p)
    rng = np.random.default_rng(0)
    n = bspline.n_functions(knots, p)
    for e in range(len(bp) - 1):
        x = rng.uniform(bp[e], bp[e + 1], size=7)
        B = bspline.local_basis(knots, p, e, x)
        D = bspline.local_basis_deriv(knots, p, e, x)
        for a in range(p + 1):
            c = np.zeros(n)
            c[e + a] = 1.0
            s = BSpline(knots, c, p)
            np.testing.assert_allclose(B[:, a], s(x), rtol=0, atol=1e-14)
            np.testing.assert_allclose(D[:, a], s.derivative()(x), rtol=0, atol=1e-11)


@pytest.mark.parametrize("kp", list(_knot_vectors()))
def test_partition_of_unity_and_integral(kp):
    knots, p = kp
    bp = bspline.breakpoints(knots, p)
    n = bspline.n_functions(knots, p)
    integ = np.zeros(n)
    for e in range(len(bp) - 1):
        x, w = gauss_on(p + 1, bp[e], bp[e + 1])
        B = bspline.local_basis(knots, p, e, x)
        np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
        integ[e:e + p + 1] += w @ B
    # int B_i = (xi_{i+p+1} - xi_i) / (p+1)
    ref = np.array([(knots[i + p + 1] - knots[i]) / (p + 1) for i in range(n)])
    np.testing.assert_allclose(integ, ref, atol=1e-15)


def test_gauss_exact_degree():
    for n in range(1, 9):
        x, w = gauss_on(n, 0.2, 0.7)
        for deg in range(2 * n):
            exact = (0.7 ** (deg + 1) - 0.2 ** (deg + 1)) / (deg + 1)
            assert abs(np.sum(w * x ** deg) - exact) < 1e-15
