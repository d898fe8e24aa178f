"""Seeded synthetic workloads: trimmed bivariate B-spline patches.

This module only *draws* inputs (knot vectors, trimming curves, geometry
control points, per-point fields and vectors). It holds none of the method's
arithmetic: no basis evaluation, no quadrature, no trimming logic. Both the
HIP path and the CPU oracle read their inputs from here.

The paper's own trim cases (line, circle, curvy corner cut; Sect. 4, Fig.
"Domains") exist only as figures, so these patches stand in for them:

* ``config1`` -- degree 2, 32x32 elements, identity geometry, c = 1, a circular
  hole of centre (0.5, 0.5) and radius 0.25, hybrid Gauss, L2 projection of
  sin(pi x) cos(pi y).
* ``config2`` -- degree 4, 256x256 elements, perturbed geometry with c = |det J|,
  a hole bounded by a closed cubic periodic B-spline with 16 control points.
* ``config3`` -- degree 6, 512x512 elements, perturbed geometry, a hole that is
  the union of three seeded ellipses.
* ``config4`` -- 256 independent patches of seeded degree 2..5 and seeded
  element counts, one elliptical hole each.
* ``config5`` -- degree 4, 1024x1024 elements, the 16-point cubic hole, and
  per-point coefficient values for the matrix-free product and its adjoint.
* ``table1_line`` -- 10x10 elements cut by a straight line (the accuracy
  experiment of Sect. 4.1, Table 1).

All draws use ``numpy.random.default_rng(seed)`` in the order documented on
each generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 210108053

CURVE_BSPLINE = 0   # closed periodic uniform B-spline, degree 1..3
CURVE_ELLIPSE = 1   # ellipse (circle when a == b)

METHOD_GAUSS_REF = 0
METHOD_HYBRID = 1
METHOD_DWQ = 2
METHOD_NAIVE_WQ = 3

COEF_CONST = 0
COEF_GEOM_DETJ = 1
COEF_AT_POINTS = 2


@dataclass
class Curve:
    """A closed trimming curve bounding one hole (the hole is its interior)."""
    kind: int
    degree: int = 3
    cp: Optional[np.ndarray] = None        # (m, 2) control points, BSPLINE
    cx: float = 0.0                        # ELLIPSE centre, semi-axes, rotation
    cy: float = 0.0
    a: float = 0.0
    b: float = 0.0
    phi: float = 0.0


@dataclass
class Patch:
    p: int
    n_el: tuple                            # (N1, N2) elements per direction
    knots: tuple                           # (knots1, knots2) open knot vectors
    curves: List[Curve] = field(default_factory=list)
    geom_cp: Optional[np.ndarray] = None   # (n2, n1, 2) control points or None
    coef: int = COEF_CONST
    coef_value: float = 1.0
    name: str = ""

    @property
    def n_fn(self):
        return (self.n_el[0] + self.p, self.n_el[1] + self.p)


def open_uniform_knots(n_el: int, p: int) -> np.ndarray:
    """Open knot vector on [0, 1] with n_el equal elements, ends repeated p+1 times."""
    inner = np.linspace(0.0, 1.0, n_el + 1)
    return np.concatenate([np.zeros(p), inner, np.ones(p)])


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    n = len(knots) - p - 1
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(n)])


def perturbed_geometry(rng, p, n_el, noise=0.1):
    """Greville grid of the patch's own space plus U[-noise*h, noise*h] per component.

    One draw of shape (n2, n1, 2), consumed from ``rng`` first.
    """
    N1, N2 = n_el
    k1, k2 = open_uniform_knots(N1, p), open_uniform_knots(N2, p)
    g1, g2 = greville(k1, p), greville(k2, p)
    n1, n2 = len(g1), len(g2)
    h = np.array([1.0 / N1, 1.0 / N2])
    delta = rng.uniform(-1.0, 1.0, size=(n2, n1, 2)) * (noise * h)
    cp = np.empty((n2, n1, 2))
    cp[..., 0] = g1[None, :]
    cp[..., 1] = g2[:, None]
    return cp + delta


def identity_geometry(p, n_el):
    N1, N2 = n_el
    g1 = greville(open_uniform_knots(N1, p), p)
    g2 = greville(open_uniform_knots(N2, p), p)
    cp = np.empty((len(g2), len(g1), 2))
    cp[..., 0] = g1[None, :]
    cp[..., 1] = g2[:, None]
    return cp


def radial_cubic_curve(rng, n_cp=16, r0=0.3, dr=0.05, centre=(0.5, 0.5)):
    """Closed cubic periodic B-spline, control points at r_k = r0 + dr*u_k, u_k ~ U[0,1].

    Angles are 2*pi*k/n_cp; one draw of n_cp uniforms.
    """
    u = rng.uniform(0.0, 1.0, size=n_cp)
    th = 2.0 * math.pi * np.arange(n_cp) / n_cp
    r = r0 + dr * u
    cp = np.stack([centre[0] + r * np.cos(th), centre[1] + r * np.sin(th)], axis=1)
    return Curve(kind=CURVE_BSPLINE, degree=3, cp=cp)


def random_ellipse(rng, axes=(0.05, 0.2), centre=(0.25, 0.75)):
    """Semi-axes ~ U[axes], centre ~ U[centre]^2, rotation ~ U[0, pi). Five draws."""
    a, b = rng.uniform(axes[0], axes[1], size=2)
    cx, cy = rng.uniform(centre[0], centre[1], size=2)
    phi = rng.uniform(0.0, math.pi)
    return Curve(kind=CURVE_ELLIPSE, cx=float(cx), cy=float(cy), a=float(a), b=float(b), phi=float(phi))


def circle(cx, cy, r):
    return Curve(kind=CURVE_ELLIPSE, cx=cx, cy=cy, a=r, b=r, phi=0.0)


def _patch(p, N1, N2, curves, geom_cp=None, coef=COEF_CONST, name=""):
    return Patch(p=p, n_el=(N1, N2), knots=(open_uniform_knots(N1, p), open_uniform_knots(N2, p)),
                 curves=curves, geom_cp=geom_cp, coef=coef, name=name)


def config1(N=32, p=2):
    """Degree 2, N x N elements, identity map (c = 1), circular hole r = 0.25."""
    return _patch(p, N, N, [circle(0.5, 0.5, 0.25)], None, COEF_CONST, f"circle_p{p}_N{N}")


def config1_target(x, y, xp=np):
    """Target of the projection in config 1: g = sin(pi x) cos(pi y)."""
    return xp.sin(math.pi * x) * xp.cos(math.pi * y)


def config2(N=256, p=4, seed=SEED_BASE + 2, n_cp=16):
    """Degree p, N x N, perturbed geometry (c = |det J|), cubic 16-point hole.

    Draw order: geometry noise (n2, n1, 2), then the n_cp radii uniforms.
    """
    rng = np.random.default_rng(seed)
    geom = perturbed_geometry(rng, p, (N, N))
    curve = radial_cubic_curve(rng, n_cp=n_cp)
    return _patch(p, N, N, [curve], geom, COEF_GEOM_DETJ, f"cubic16_p{p}_N{N}")


def config3(N=512, p=6, seed=SEED_BASE + 3, n_ell=3):
    """Degree p, N x N, perturbed geometry, hole = union of n_ell seeded ellipses.

    Draw order: geometry noise, then per ellipse (a, b), (cx, cy), phi.
    """
    rng = np.random.default_rng(seed)
    geom = perturbed_geometry(rng, p, (N, N))
    curves = [random_ellipse(rng) for _ in range(n_ell)]
    return _patch(p, N, N, curves, geom, COEF_GEOM_DETJ, f"ellipses{n_ell}_p{p}_N{N}")


def config4(n_patch=256, seed=SEED_BASE + 4, n_range=(16, 256), p_range=(2, 5)):
    """n_patch independent patches: p ~ U{2..5}, N_d = round(exp(U[ln 16, ln 256])).

    Draw order per patch: p, (N1, N2) log-uniforms, geometry noise, one ellipse.
    """
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_patch):
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        lo, hi = math.log(n_range[0]), math.log(n_range[1])
        N1, N2 = (int(round(math.exp(v))) for v in rng.uniform(lo, hi, size=2))
        geom = perturbed_geometry(rng, p, (N1, N2))
        ell = random_ellipse(rng)
        out.append(_patch(p, N1, N2, [ell], geom, COEF_GEOM_DETJ, f"batch{k}_p{p}_{N1}x{N2}"))
    return out


def config5(N=1024, p=4, seed=SEED_BASE + 5):
    """Matrix-free workload: degree p, N x N, identity map, 16-point cubic hole.

    Draw order: the n_cp radii uniforms. Vectors u, f are drawn later with
    ``config5_vectors`` once the number of active functions is known.
    """
    rng = np.random.default_rng(seed)
    curve = radial_cubic_curve(rng)
    return _patch(p, N, N, [curve], None, COEF_AT_POINTS, f"mf_cubic16_p{p}_N{N}")


def config5_coef(x, y, xp=np):
    """Per-point coefficient of config 5: c = 1 + 0.5 sin(2 pi x) sin(2 pi y)."""
    return 1.0 + 0.5 * xp.sin(2.0 * math.pi * x) * xp.sin(2.0 * math.pi * y)


def config5_vectors(n_act, seed=SEED_BASE + 50):
    """u ~ N(0,1) and f ~ N(0,1) of length n_act (drawn in that order)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(n_act)
    f = rng.standard_normal(n_act)
    return u, f


def table1_line(p, N=10, y0=0.31, y1=0.67):
    """N x N elements cut by the straight line from (0, y0) to (1, y1).

    The hole is the part of the plane above the line, bounded by a closed
    polygon (a degree-1 periodic B-spline) that reaches beyond the unit square.
    """
    s = (y1 - y0)
    yl, yr = y0 - 0.5 * s, y1 + 0.5 * s
    cp = np.array([[-0.5, yl], [1.5, yr], [1.5, 2.0], [-0.5, 2.0]])
    return _patch(p, N, N, [Curve(kind=CURVE_BSPLINE, degree=1, cp=cp)], None, COEF_CONST,
                  f"line_p{p}_N{N}")


def nonuniform_knots(rng, n_el: int, p: int, jitter=0.3) -> np.ndarray:
    """Open knot vector on [0, 1] with simple interior knots k/n_el + U[-jitter h, jitter h] (h = 1/n_el).

    One draw of n_el - 1 uniforms; the knots stay increasing for jitter < 0.5.
    """
    h = 1.0 / n_el
    inner = np.arange(1, n_el) * h + rng.uniform(-jitter, jitter, size=n_el - 1) * h
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def nonuniform_variant(cfg, seed=SEED_BASE + 7, jitter=0.3):
    """The same patch (degree, element counts, curves, geometry, coefficient) on non-uniform knots.

    Draw order: direction-1 knots, then direction-2 knots. The geometry's control points are kept
    (one per function), so a perturbed geometry stays a valid map of the new space.
    """
    rng = np.random.default_rng(seed)
    k1 = nonuniform_knots(rng, cfg.n_el[0], cfg.p, jitter)
    k2 = nonuniform_knots(rng, cfg.n_el[1], cfg.p, jitter)
    return Patch(p=cfg.p, n_el=cfg.n_el, knots=(k1, k2), curves=cfg.curves, geom_cp=cfg.geom_cp, coef=cfg.coef,
                 coef_value=cfg.coef_value, name=cfg.name + "_nonuniform")


def small_variant(cfg_fn, N, p=None, **kw):
    """Same generator at a smaller element count (for parity tests)."""
    if p is None:
        return cfg_fn(N=N, **kw)
    return cfg_fn(N=N, p=p, **kw)
