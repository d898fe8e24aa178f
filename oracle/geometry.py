"""Pull-back coefficient c of the mass integrand (Sect. 2.1: c is set by the geometry map).

For a B-spline map F(xi) = sum_ij P_ij B_i(xi_1) B_j(xi_2) of the patch's own
space, c = |det DF| turns the physical mass integral into Eq. (6) on the
parameter domain. Physical points F(xi) are needed to evaluate a target
function in the L2 projection.
"""
from __future__ import annotations

import numpy as np

from . import bspline


def _group_by_element(bp1, bp2, x, y, e1=None, e2=None):
    if e1 is None:
        e1 = bspline.element_of(bp1, x)
    if e2 is None:
        e2 = bspline.element_of(bp2, y)
    return np.asarray(e1), np.asarray(e2)


def map_and_detj(patch, x, y, e1=None, e2=None):
    """Physical coordinates (X, Y) and det DF at parameter points (x, y)."""
    p = patch.p
    k1, k2 = patch.knots
    bp1, bp2 = bspline.breakpoints(k1, p), bspline.breakpoints(k2, p)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    e1, e2 = _group_by_element(bp1, bp2, x, y, e1, e2)
    e1 = np.broadcast_to(e1, x.shape)
    e2 = np.broadcast_to(e2, x.shape)
    X = np.empty_like(x)
    Y = np.empty_like(x)
    D = np.empty_like(x)
    P = patch.geom_cp
    keys = e2.astype(np.int64) * (len(bp1) - 1) + e1
    for key in np.unique(keys):
        idx = np.nonzero(keys == key)[0]
        a1, a2 = int(e1[idx[0]]), int(e2[idx[0]])
        B1 = bspline.local_basis(k1, p, a1, x[idx])
        D1 = bspline.local_basis_deriv(k1, p, a1, x[idx])
        B2 = bspline.local_basis(k2, p, a2, y[idx])
        D2 = bspline.local_basis_deriv(k2, p, a2, y[idx])
        blk = P[a2:a2 + p + 1, a1:a1 + p + 1, :]          # [j2, j1, comp]
        X[idx] = np.einsum("gi,gj,ji->g", B1, B2, blk[..., 0])
        Y[idx] = np.einsum("gi,gj,ji->g", B1, B2, blk[..., 1])
        x1 = np.einsum("gi,gj,ji->g", D1, B2, blk[..., 0])
        x2 = np.einsum("gi,gj,ji->g", B1, D2, blk[..., 0])
        y1 = np.einsum("gi,gj,ji->g", D1, B2, blk[..., 1])
        y2 = np.einsum("gi,gj,ji->g", B1, D2, blk[..., 1])
        D[idx] = x1 * y2 - x2 * y1
    return X, Y, D


class Coefficient:
    """c at parameter points: constant, |det DF| of the patch geometry, or a given field.

    ``field(x, y)`` (parameter coordinates) stands for per-point data.
    """

    def __init__(self, patch, kind=None, value=1.0, field=None):
        from paper_2101_08053_amd import workloads as wl
        self.patch = patch
        self.kind = patch.coef if kind is None else kind
        self.value = value
        self.field = field
        self.wl = wl

    def __call__(self, x, y, e1=None, e2=None):
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        y = np.atleast_1d(np.asarray(y, dtype=np.float64))
        if self.kind == self.wl.COEF_CONST:
            return np.full(np.broadcast(x, y).shape, float(self.value))
        if self.kind == self.wl.COEF_GEOM_DETJ:
            return np.abs(map_and_detj(self.patch, x, y, e1, e2)[2])
        if self.kind == self.wl.COEF_AT_POINTS:
            return self.field(x, y)
        raise ValueError("unknown coefficient kind")

    def physical(self, x, y, e1=None, e2=None):
        if self.patch.geom_cp is None:
            return np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
        X, Y, _ = map_and_detj(self.patch, x, y, e1, e2)
        return X, Y
