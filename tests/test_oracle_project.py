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
    # M over all functions (exterior included) applied to the coefficients
    ref = o.gauss_reference().toarray() @ coeffs[o.ts.active]
    # exterior functions vanish on the visible domain, so dropping them changes nothing
    np.testing.assert_allclose(br, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(bh, ref, rtol=0, atol=1e-14)


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
