"""Pins of the oracle's extended B-spline stabilisation (CPU).

* the extension weights reproduce polynomials: with the coefficients c of a
  polynomial in the full basis (fitted independently by least squares on
  SciPy's B-spline design matrix), E^T c_inner = c on every outer function,
  on uniform and non-uniform knots;
* on uniform knots away from the repeated ends the 1-D weights are the
  Lagrange extrapolation weights of the nodes l..l+p at j (the coefficients
  of a polynomial are a polynomial of the same degree in the index there),
  to 1e-13, also on fine meshes where the monomial conditions are
  ill-conditioned in floating point;
* the extended projection reproduces Q_p on trimmed patches;
* on a sliver trim the extended matrix is far better conditioned than the
  plain one, and the projection error stays that of the plain projection.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import extended, project
from oracle.assemble import Oracle
from oracle.geometry import Coefficient
from paper_2101_08053_amd import workloads as wl


def _const(cfg):
    cfg.geom_cp = None
    return Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_CONST))


def _sliver(p, N=10, y=0.505):
    """A horizontal line leaving a strip of height 0.005 of the row of elements above y = 0.5."""
    return wl.table1_line(p, N=N, y0=y, y1=y)


def _coeffs_1d(knots, p, q):
    """Coefficients of the polynomial q in the B-spline basis: least squares on many points."""
    n = len(knots) - p - 1
    x = np.linspace(knots[0], knots[-1], 8 * n + 7)
    A = BSpline.design_matrix(x, knots, p).toarray()
    c, *_ = np.linalg.lstsq(A, q(x), rcond=None)
    return c


@pytest.mark.parametrize("cfg", [_sliver(3), wl.config1(N=16, p=2), wl.nonuniform_variant(wl.config1(N=14, p=3))],
                         ids=lambda c: c.name)
def test_extension_reproduces_polynomials(cfg):
    o = _const(cfg)
    inner_flat, E = extended.extension(o)
    ts, p = o.ts, o.p
    assert E.shape[0] < ts.n_act   # some functions are outer
    for a in range(p + 1):
        for b in range(p + 1):
            c1 = _coeffs_1d(o.k1, p, lambda x: x ** a)
            c2 = _coeffs_1d(o.k2, p, lambda y: y ** b)
            c = np.outer(c2, c1).reshape(-1)[ts.active]          # coefficient of B_(i1,i2) = c1[i1] c2[i2]
            ci = np.outer(c2, c1).reshape(-1)[inner_flat]
            err = np.abs(E.T @ ci - c).max()
            assert err <= 1e-11 * max(1.0, np.abs(c).max()), (a, b, err)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("N", [16, 1024])
def test_weights_are_lagrange_extrapolation(p, N):
    knots = np.r_[np.zeros(p), np.linspace(0.0, 1.0, N + 1), np.ones(p)]
    n = N + p
    worst, seen = 0.0, 0
    for j, l in [(n // 2, n // 2 + 1), (n // 2, n // 2 - p - 3), (n // 2 + 2, n // 2 - p), (n // 2 - 4, n // 2),
                 (p - 1, p), (2 * p, p - 1)]:
        if min(j, l) + 1 < p or max(j, l + p) + p > p + N:
            continue   # reads a repeated end knot
        e = extended.weights_1d(knots, p, j, l)
        lag = np.array([np.prod([(j - (l + k)) / (m - k) for k in range(p + 1) if k != m]) for m in range(p + 1)])
        worst = max(worst, np.abs(e - lag).max() / max(1.0, np.abs(lag).max()))
        seen += 1
    assert seen >= 2 and worst <= 1e-13, (seen, worst)


@pytest.mark.parametrize("cfg", [_sliver(3), wl.config1(N=12), wl.config3(N=12, p=4)], ids=lambda c: c.name)
def test_extended_projection_reproduces_qp(cfg):
    o = _const(cfg)
    p = cfg.p

    def g(x, y):
        return x ** p * y ** (p - 1) - 0.5 * x * y ** p + 0.25

    _, E = extended.extension(o)
    u = extended.solve_extended(o.hybrid(), project.rhs(o, g), E)
    assert project.l2_error(o, u, g) < 1e-10


def test_extension_conditions_a_sliver():
    o = _const(_sliver(3))
    M = o.hybrid()
    _, E = extended.extension(o)
    A = (0.5 * (M + M.T)).toarray()
    Ae = E @ A @ E.T
    cond = np.linalg.cond(A)
    cond_e = np.linalg.cond(np.asarray(Ae))
    assert cond > 1e6 and cond_e < 1e-3 * cond, (cond, cond_e)
    b = project.rhs(o, wl.config1_target)
    u = project.solve(M, b)
    ue = extended.solve_extended(M, b, E)
    e0 = project.l2_error(o, u, wl.config1_target)
    e1 = project.l2_error(o, ue, wl.config1_target)
    assert e1 <= 2.0 * e0 + 1e-12, (e0, e1)
