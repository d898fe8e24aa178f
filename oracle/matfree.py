"""Matrix-free product y = M(c) u and its gradient, as explicit sparse operators.

With c a value per rule point, every row rule reads
    y_i = sum_k w_hat_{k,i} c_k (B u)_k,
so M(c) = What diag(c) Bmat with What[i, k] = row i's test-side weight at
point k (w1 w2 for weighted-quadrature rows, w_g B_i(x_g) for element-formed
rows) and Bmat[k, j] = B_j(x_k). For L = 1/2 ||M(c) u - f||^2, r = M(c) u - f:
    dL/du = M(c)^T r = Bmat^T diag(c) What^T r,   dL/dc = (Bmat u) * (What^T r).
Points are ordered as the library orders them: the WQ grid (k2 outer), then
(p+1)^2 Gauss points per band element (flat element order, g2 outer), then
the cut-element nodes (cut elements in flat order).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import bspline


def rule_points(o):
    """(x, y, e1, e2) of every rule point of the hybrid rules, in the library's order."""
    ts = o.ts
    Q1, Q2 = len(o.xs1), len(o.xs2)
    xs = [np.tile(o.xs1, Q2)]
    ys = [np.repeat(o.xs2, Q1)]
    e1s = [np.tile(o.el1, Q2)]
    e2s = [np.repeat(o.el2, Q1)]
    ws = [np.zeros(Q1 * Q2)]
    for (e1, e2) in ts.band_elements():
        x, y, w = o.element_points(e1, e2)
        xs.append(x), ys.append(y), ws.append(w)
        e1s.append(np.full(len(x), e1)), e2s.append(np.full(len(x), e2))
    for (e1, e2) in ts.cut_elements():
        x, y, w, _ = ts.cut_rule(e1, e2)
        xs.append(x), ys.append(y), ws.append(w)
        e1s.append(np.full(len(x), e1)), e2s.append(np.full(len(x), e2))
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(e1s).astype(np.int64),
            np.concatenate(e2s).astype(np.int64), np.concatenate(ws))


def operators(o):
    """What (n_act x n_pts) and Bmat (n_pts x n_act) of the hybrid rules."""
    ts = o.ts
    p = o.p
    x, y, e1, e2, wg = rule_points(o)
    npts = len(x)
    Q1 = len(o.xs1)
    # Bmat
    R, C, V = [], [], []
    keys = e2 * ts.N1 + e1
    for key in np.unique(keys):
        idx = np.nonzero(keys == key)[0]
        a1, a2 = int(e1[idx[0]]), int(e2[idx[0]])
        B1 = bspline.local_basis(o.k1, p, a1, x[idx])
        B2 = bspline.local_basis(o.k2, p, a2, y[idx])
        for b2 in range(p + 1):
            for b1 in range(p + 1):
                col = ts.act_of[(a2 + b2) * ts.n1 + a1 + b1]
                if col >= 0:
                    R.append(idx)
                    C.append(np.full(len(idx), col))
                    V.append(B1[:, b1] * B2[:, b2])
    Bmat = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(npts, ts.n_act))
    # What
    R, C, V = [], [], []
    for f in o.interior_rows_flat():
        i2, i1 = divmod(int(f), ts.n1)
        q1 = np.nonzero(o.W1[i1])[0]
        q2 = np.nonzero(o.W2[i2])[0]
        k = (q2[None, :] * Q1 + q1[:, None]).ravel()
        w = np.outer(o.W1[i1, q1], o.W2[i2, q2]).ravel()
        R.append(np.full(len(k), ts.act_of[f]))
        C.append(k)
        V.append(w)
    elem_rows = np.zeros(ts.n1 * ts.n2, dtype=bool)
    elem_rows[o.cut_rows_flat()] = True
    n_wq = len(o.xs1) * len(o.xs2)
    sel = np.arange(npts) >= n_wq
    for key in np.unique(keys[sel]):
        idx = np.nonzero((keys == key) & sel)[0]
        a1, a2 = int(e1[idx[0]]), int(e2[idx[0]])
        B1 = bspline.local_basis(o.k1, p, a1, x[idx])
        B2 = bspline.local_basis(o.k2, p, a2, y[idx])
        for b2 in range(p + 1):
            for b1 in range(p + 1):
                f = (a2 + b2) * ts.n1 + a1 + b1
                if elem_rows[f]:
                    R.append(np.full(len(idx), ts.act_of[f]))
                    C.append(idx)
                    V.append(wg[idx] * B1[:, b1] * B2[:, b2])
    What = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(ts.n_act, npts))
    return What, Bmat


def apply(What, Bmat, c, u):
    return What @ (c * (Bmat @ u))


def gradient(What, Bmat, c, u, f):
    """L = 1/2 ||M(c) u - f||^2: returns (L, dL/du, dL/dc)."""
    r = apply(What, Bmat, c, u) - f
    R = What.T @ r
    return 0.5 * float(r @ r), Bmat.T @ (c * R), (Bmat @ u) * R
