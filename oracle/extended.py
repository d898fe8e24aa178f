"""Extended B-spline stabilisation of the trimmed basis.

Test infrastructure: plain and slow, written for checking the device path;
nothing here is used by the library.

The paper applies the extended B-spline concept to every L2 projection
(Sect. 2.2, last paragraph, and Sect. 4.2) to keep the mass matrix well
conditioned when the trimming curve leaves only a sliver of a function's
support, and refers to the literature for the construction. Restated here
(weighted extended B-splines without weight function, the trimmed patch's
B-splines themselves):

* an active function is inner if its support holds an inside element, outer
  otherwise (only cut elements of it are visible);
* every outer function j is tied to a block I(j) = {l1..l1+p} x {l2..l2+p}
  of (p+1)^2 inner functions near it;
* per direction the weights e_m (m = 0..p) make the block reproduce the
  outer function's coefficient of every polynomial of degree <= p. The
  coefficient of a polynomial q in the B-spline basis is the dual functional
  lambda_i(q); on monomials lambda_i(x^k) = sigma_k(t_{i+1}, ..., t_{i+p}) /
  binom(p, k), sigma_k the elementary symmetric polynomial of the knots
  inside B_i's support (Marsden's identity), so the weights solve
      sum_m e_m lambda_{l+m}(x^k) = lambda_j(x^k),  k = 0..p
  (on uniform knots away from the ends: Lagrange extrapolation of the
  coefficient sequence from the nodes l..l+p to j), here in exact rational
  arithmetic;
* e_{i,j} = e^1_{i1 - l1}(j1) e^2_{i2 - l2}(j2), and the extended basis is
  B_i^e = B_i + sum_{outer j : i in I(j)} e_{i,j} B_j over the inner i.
  With E[i, j] = 1 (j = i inner) or e_{i,j} (j outer, i in I(j)) the
  projection solves (E A E^T) u_e = E b and returns u = E^T u_e.

Block choice (a reading: the paper does not fix one): among the blocks whose
(p+1)^2 functions are all inner, the one whose centre (l + p/2) is nearest
to j in the Euclidean index distance; ties go to the smaller l2, then the
smaller l1.
"""
from __future__ import annotations

import math
from fractions import Fraction
from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .trim import INSIDE


def inner_mask(ts):
    """[n2, n1] bool: active functions whose support holds an inside element."""
    p = ts.p
    out = np.zeros((ts.n2, ts.n1), dtype=bool)
    for i2 in range(ts.n2):
        for i1 in range(ts.n1):
            sub = ts.ecls[max(0, i2 - p):min(ts.N2, i2 + 1), max(0, i1 - p):min(ts.N1, i1 + 1)]
            out[i2, i1] = bool(np.any(sub == INSIDE))
    return out


def weights_1d(knots, p, j, l):
    """e_m, m = 0..p: the block l..l+p reproduces B_j's coefficient of every polynomial of degree p.

    The conditions sum_m e_m lambda_{l+m}(x^k) = lambda_j(x^k), k = 0..p, are solved in exact
    rational arithmetic from the (exactly representable) floating-point knots: in floating point
    their condition number grows with the distance from j to the block and with p (about 1e7 at
    p = 8 even on centred, scaled monomials), the exact solution has none of that error.
    """
    t = [Fraction(float(x)) for x in knots]

    def lam(i, k):
        s = sum((math.prod(c) for c in combinations(t[i + 1:i + p + 1], k)), Fraction(0)) if k > 0 else Fraction(1)
        return s / math.comb(p, k)

    n = p + 1
    A = [[lam(l + m, k) for m in range(n)] + [lam(j, k)] for k in range(n)]
    for c in range(n):   # Gauss-Jordan elimination, exact
        r = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[r] = A[r], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [a - f * b for a, b in zip(A[r], A[c])]
    return np.array([float(A[r][n] / A[r][r]) for r in range(n)])


def all_inner_blocks(inner, p):
    """[n2 - p, n1 - p] bool: blocks {l1..l1+p} x {l2..l2+p} whose functions are all inner."""
    n2, n1 = inner.shape
    ok = np.zeros((n2 - p, n1 - p), dtype=bool)
    for l2 in range(n2 - p):
        for l1 in range(n1 - p):
            ok[l2, l1] = inner[l2:l2 + p + 1, l1:l1 + p + 1].all()
    return ok


def choose_block(ok, j1, j2, p):
    """(l1, l2) of the all-inner block nearest to j (centre l + p/2), or None.

    Distances are compared as integers, d = (2 l1 + p - 2 j1)^2 + (2 l2 + p - 2 j2)^2,
    ties to the smaller l2, then l1. Windows of blocks whose centre lies within R of j
    in each coordinate grow until the best one found is within R (so none outside is nearer).
    """
    nb2, nb1 = ok.shape
    if not ok.any():
        return None
    R = p
    while True:
        best = None
        lo1, hi1 = max(0, math.ceil(j1 - p / 2 - R)), min(nb1 - 1, math.floor(j1 - p / 2 + R))
        lo2, hi2 = max(0, math.ceil(j2 - p / 2 - R)), min(nb2 - 1, math.floor(j2 - p / 2 + R))
        for l2 in range(lo2, hi2 + 1):
            for l1 in range(lo1, hi1 + 1):
                if ok[l2, l1]:
                    key = ((2 * l1 + p - 2 * j1) ** 2 + (2 * l2 + p - 2 * j2) ** 2, l2, l1)
                    if best is None or key < best:
                        best = key
        if best is not None and best[0] <= 4 * R * R:
            return best[2], best[1]
        R = 2 * R if best is None else max(2 * R, math.ceil(math.sqrt(best[0]) / 2))


def extension(o):
    """(inner flat indices, E) with E sparse [n_inner x n_act] over the plan's compact rows."""
    ts, p = o.ts, o.p
    inner = inner_mask(ts) & (ts.act_of.reshape(ts.n2, ts.n1) >= 0)
    ok = all_inner_blocks(inner, p)
    inner_flat = [int(f) for f in np.nonzero(inner.reshape(-1))[0]]
    row_of = {f: r for r, f in enumerate(inner_flat)}
    R, C, V = [], [], []
    for f in ts.active:
        f = int(f)
        c = int(ts.act_of[f])
        if f in row_of:
            R.append(row_of[f])
            C.append(c)
            V.append(1.0)
            continue
        i2, i1 = divmod(f, ts.n1)
        blk = choose_block(ok, i1, i2, p)
        if blk is None:
            raise ValueError("no block of inner functions")
        l1, l2 = blk
        w1 = weights_1d(o.k1, p, i1, l1)
        w2 = weights_1d(o.k2, p, i2, l2)
        for m2 in range(p + 1):
            for m1 in range(p + 1):
                R.append(row_of[(l2 + m2) * ts.n1 + (l1 + m1)])
                C.append(c)
                V.append(w1[m1] * w2[m2])
    E = sp.csr_matrix((V, (R, C)), shape=(len(inner_flat), ts.n_act))
    return inner_flat, E


def solve_extended(M, b, E):
    """u = E^T u_e with (E A E^T) u_e = E b, A = (M + M^T)/2."""
    A = 0.5 * (M + M.T)
    Ae = (E @ A @ E.T).tocsc()
    ue = spla.spsolve(Ae, E @ b)
    return E.T @ ue
