"""Pins of the oracle's L2 projection and matrix-free gradient (CPU)."""
import math

import numpy as np
import pytest

from oracle import bspline, matfree, project
from oracle.assemble import Oracle
from oracle.geometry import Coefficient
from paper_2101_08053_amd import workloads as wl


def _const(cfg):
    return Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_CONST))


@pytest.mark.parametrize("cfg", [wl.config1(N=12), wl.table1_line(3), wl.config2(N=10, p=2)],
                         ids=lambda c: c.name)
def test_polynomial_reproduction(cfg):
    """g in Q_p (identity map, c = 1): the projection reproduces g (Sect. 4.2)."""
    cfg.geom_cp = None
    o = _const(cfg)
    p = cfg.p

    def g(x, y):
        return x ** p * y ** p - 0.5 * x ** (p - 1) * y + 0.25

    M = o.hybrid()
    b = project.rhs(o, g)
    u = project.solve(M, b)
    assert project.l2_error(o, u, g) < 1e-10


def test_rate_p_plus_1():
    """Relative L2 error of sin(pi x) cos(pi y) on the circle-trimmed patch drops at order p+1."""
    errs = []
    Ns = (8, 16, 32)
    for N in Ns:
        cfg = wl.config1(N=N)
        o = _const(cfg)
        u = project.solve(o.hybrid(), project.rhs(o, wl.config1_target))
        errs.append(project.l2_error(o, u, wl.config1_target))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert rates[-1] > 2.7, (errs, rates)


def test_reference_and_hybrid_rhs_agree_for_splines():
    """For g in the spline space both rules are exact, so b is M g_coeffs."""
    cfg = wl.config1(N=10)
    o = _const(cfg)
    rng = np.random.default_rng(5)
    coeffs = rng.standard_normal(o.ts.n1 * o.ts.n2)

    def g(x, y):
        out = np.zeros_like(x)
        e1 = bspline.element_of(o.ts.bp1, x)
        e2 = bspline.element_of(o.ts.bp2, y)
        for k in range(len(x)):
            B1 = bspline.local_basis(o.k1, o.p, int(e1[k]), x[k:k + 1])[0]
            B2 = bspline.local_basis(o.k2, o.p, int(e2[k]), y[k:k + 1])[0]
            blk = coeffs.reshape(o.ts.n2, o.ts.n1)[e2[k]:e2[k] + o.p + 1, e1[k]:e1[k] + o.p + 1]
            out[k] = B2 @ blk @ B1
        return out

    bh = project.rhs(o, g, "hybrid")
    br = project.rhs(o, g, "reference")
    bd = project.rhs(o, g, "dwq")
    # M over all functions (exterior included) applied to the coefficients
    ref = o.gauss_reference().toarray() @ coeffs[o.ts.active]
    # exterior functions vanish on the visible domain, so dropping them changes nothing
    np.testing.assert_allclose(br, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(bh, ref, rtol=0, atol=1e-14)
    # the refined weights integrate B_i B_j exactly on their box (Sect. 3.3), hence any spline g
    np.testing.assert_allclose(bd, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("cfg", [wl.table1_line(3), wl.config1(N=12), wl.config3(N=14, p=4)],
                         ids=lambda c: c.name)
def test_dwq_rhs_boxes_and_polynomial_reproduction(cfg):
    """DWQ matrix and right-hand side: g in Q_p is reproduced (identity map, c = 1, Sect. 4.2)."""
    cfg.geom_cp = None
    o = _const(cfg)
    p = cfg.p
    n_box = sum(o.dwq_region(int(f) % o.ts.n1, int(f) // o.ts.n1) is not None for f in o.cut_rows_flat())
    assert n_box > 0   # some cut rows do take their box part from the refined weights

    def g(x, y):
        return x ** p * y ** (p - 1) - 0.5 * x * y ** p + 0.25

    u = project.solve(o.dwq(), project.rhs(o, g, "dwq"))
    assert project.l2_error(o, u, g) < 1e-10


def test_dwq_rhs_of_one_is_the_row_sum():
    """g = 1: b_i = sum_j M_ij of the DWQ matrix (the B_j sum to one on the visible domain), mapped
    geometry with c = |det J| evaluated at the nested points."""
    cfg = wl.config2(N=12, p=3)
    o = Oracle(cfg)
    b = project.rhs(o, lambda x, y: np.ones_like(x), "dwq")
    Sb = project.rhs(o, lambda x, y: np.ones_like(x), "dwq", absolute=True)
    rows = np.asarray(o.dwq().sum(axis=1)).ravel()
    assert np.abs(b - rows).max() <= 1e-13 * Sb.max()
    # the cut rows differ from the hybrid rule's (the boxes change their quadrature)
    bh = project.rhs(o, lambda x, y: np.ones_like(x), "hybrid")
    cut = o.ts.act_of[np.asarray(o.cut_rows_flat())]
    assert np.abs(b[cut] - bh[cut]).max() > 1e-12 * Sb.max()


@pytest.mark.parametrize("cfg", [wl.config1(N=10), wl.config5(N=12)], ids=lambda c: c.name)
def test_matfree_operator_equals_formed_matrix(cfg):
    """What diag(c) Bmat reproduces the per-entry hybrid matrix for the same c."""
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_AT_POINTS, field=wl.config5_coef))
    What, Bmat = matfree.operators(o)
    x, y, *_ = matfree.rule_points(o)
    c = wl.config5_coef(x, y)
    M_op = (What @ (np.diag(c) @ Bmat.toarray()))
    M = o.hybrid().toarray()
    assert np.abs(M_op - M).max() <= 1e-13 * np.abs(M).max()


def test_matfree_gradient_finite_differences():
    """dL/du and dL/dc against central differences on a 16x16-element instance.

    L is quadratic in u and in c separately, so central differences carry no
    truncation error; the step h = 0.1 keeps cancellation in L (~1e2) at ~1e-13.
    """
    cfg = wl.config5(N=16)
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_AT_POINTS, field=wl.config5_coef))
    What, Bmat = matfree.operators(o)
    x, y, *_ = matfree.rule_points(o)
    c = wl.config5_coef(x, y)
    u, f = wl.config5_vectors(o.ts.n_act)
    L, du, dc = matfree.gradient(What, Bmat, c, u, f)
    rng = np.random.default_rng(1)
    h = 0.1
    for _ in range(3):
        v = rng.standard_normal(len(u))
        fd = (matfree.gradient(What, Bmat, c, u + h * v, f)[0] - matfree.gradient(What, Bmat, c, u - h * v, f)[0]) / (2 * h)
        assert abs(fd - du @ v) <= 1e-7 * abs(fd)
        w = rng.standard_normal(len(c))
        fd = (matfree.gradient(What, Bmat, c + h * w, u, f)[0] - matfree.gradient(What, Bmat, c - h * w, u, f)[0]) / (2 * h)
        assert abs(fd - dc @ w) <= 1e-7 * abs(fd)
    for k in rng.choice(len(u), 4, replace=False):
        e = np.zeros(len(u))
        e[k] = h
        fd = (matfree.gradient(What, Bmat, c, u + e, f)[0] - matfree.gradient(What, Bmat, c, u - e, f)[0]) / (2 * h)
        assert abs(fd - du[k]) <= 1e-7 * max(abs(fd), 1e-3)


def _disk_moment(poly, xs, ys, cx, cy, r):
    """Exact integral of a polynomial in (xs, ys) over the disk |(x, y) - (cx, cy)| <= r (polar coordinates)."""
    import sympy as sym
    rho, th = sym.symbols("rho theta", nonnegative=True)
    f = sym.expand(poly.subs({xs: cx + rho * sym.cos(th), ys: cy + rho * sym.sin(th)}) * rho)
    return sym.integrate(sym.integrate(f, (th, 0, 2 * sym.pi)), (rho, 0, r))


def _visible_integral(poly, xs, ys, cx, cy, r):
    """Exact integral over [0,1]^2 minus the disk (the disk lies inside the square)."""
    import sympy as sym
    sq = sym.integrate(sym.integrate(sym.expand(poly), (xs, 0, 1)), (ys, 0, 1))
    return sq - _disk_moment(poly, xs, ys, cx, cy, r)


def test_l2_error_closed_form_identity_map():
    """l2_error's value against an exact integral (Sect. 4.2's relative L2 error).

    Identity map, c = 1, circular hole r = 1/4: the spline with coefficients at
    the Greville abscissae in xi_1 is u_h = x on the visible domain (exterior
    functions vanish there), so with g = 1 + x y + y^2 the error is
    sqrt(int (x - g)^2 / int g^2) over the square minus the disk, computed
    exactly by SymPy. A dropped hole, a wrong rule or a missing square root
    changes the value far beyond the tolerance.
    """
    import sympy as sym
    cfg = wl.config1(N=12, p=2)
    o = _const(cfg)
    g1 = wl.greville(o.k1, o.p)
    flat = np.asarray(o.ts.active)
    u = g1[flat % o.ts.n1]

    def g(x, y):
        return 1.0 + x * y + y ** 2

    xs, ys = sym.symbols("x y")
    r, c0 = sym.Rational(1, 4), sym.Rational(1, 2)
    G = 1 + xs * ys + ys ** 2
    num = _visible_integral((xs - G) ** 2, xs, ys, c0, c0, r)
    den = _visible_integral(G ** 2, xs, ys, c0, c0, r)
    exact = float(sym.sqrt(num / den).evalf(30))
    got = project.l2_error(o, u, g)
    assert abs(got - exact) <= 1e-12 * exact, (got, exact)


def test_l2_error_closed_form_mapped():
    """l2_error with a non-affine geometry map: c = |det J| varies and g is taken at physical points.

    F(xi) = (xi1 + xi1 xi2 / 5, xi2 + xi1 / 10) is represented exactly by the
    patch's space (tensor products of the Greville abscissae are the
    B-spline coefficients of xi1 xi2), det J = 1 + xi2/5 - xi1/50 > 0. With
    u_h = 1 (all coefficients one) and g(X, Y) = X Y:
    error^2 = int c (1 - X Y)^2 / int c (X Y)^2 over the parameter domain
    minus the disk, exact by SymPy. A norm without c, or g at parameter
    instead of physical points, fails.
    """
    import sympy as sym
    p, N = 3, 10
    base = wl.config1(N=N, p=p)
    k1, k2 = base.knots
    g1, g2 = wl.greville(k1, p), wl.greville(k2, p)
    cp = np.empty((len(g2), len(g1), 2))
    cp[..., 0] = g1[None, :] + 0.2 * g1[None, :] * g2[:, None]
    cp[..., 1] = g2[:, None] + 0.1 * g1[None, :]
    cfg = wl.Patch(p=p, n_el=(N, N), knots=(k1, k2), curves=base.curves, geom_cp=cp, coef=wl.COEF_GEOM_DETJ,
                   name="mapped")
    o = Oracle(cfg)
    u = np.ones(o.ts.n_act)

    def g(X, Y):
        return X * Y

    xs, ys = sym.symbols("x y")
    X = xs + xs * ys / 5
    Y = ys + xs / 10
    detj = sym.diff(X, xs) * sym.diff(Y, ys) - sym.diff(X, ys) * sym.diff(Y, xs)
    r, c0 = sym.Rational(1, 4), sym.Rational(1, 2)
    num = _visible_integral(detj * (1 - X * Y) ** 2, xs, ys, c0, c0, r)
    den = _visible_integral(detj * (X * Y) ** 2, xs, ys, c0, c0, r)
    exact = float(sym.sqrt(num / den).evalf(30))
    got = project.l2_error(o, u, g)
    assert abs(got - exact) <= 1e-12 * exact, (got, exact)
