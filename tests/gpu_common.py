"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the oracle)."""
import sys

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_08053_amd import igatrim
    igatrim.lib()  # raises if the library is missing: no silent fallback
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def parity_metric(gpu, ref):
    """max |dM| / max(|M_ij|, 1e-3 * row max) over the band layout (slot-major)."""
    rowmax = np.abs(ref).max(axis=0, keepdims=True)
    den = np.maximum(np.abs(ref), 1e-3 * rowmax)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(gpu - ref) / den))


EPS = np.finfo(np.float64).eps


FLOOR_P3 = 1e-5
ROWFLOOR_P3 = 1e-3


def inject_oracle_rules(plan, o):
    """Give the device the oracle's rules: WQ weights of both directions and the cut nodes."""
    import torch
    for d in range(2):
        from paper_2101_08053_amd import igatrim
        qmax = plan.table(igatrim.TABLE_WQ_WEIGHTS, d).shape[1]
        plan.set_weights(d, torch.as_tensor(oracle_weight_table(o, d, qmax), device="cuda"))
    x, y, w = oracle_cut_nodes(o)
    assert len(w) == plan.sizes["n_cut_nodes"], "cut-node counts differ between the device and the oracle"
    if len(w):
        plan.set_cut_nodes(*(torch.as_tensor(v, device="cuda") for v in (x, y, w)))


def parity_S(gpu, ref, S, ts=None, label="", floor=0.0, rowfloor=0.0):
    """max |dM_ij| / max(S_ij, floor max|M|), S_ij = sum of |w c B_i B_j| over the entry's terms.

    S_ij is the scale of the rounding error of the entry's own sum (it equals
    |M_ij| when no term cancels). Under identical rules (weights and nodes
    injected from the oracle) no floor is used. End to end (the device's own
    rules) entries below ``floor`` times the largest one, or ``rowfloor`` times
    their row's largest term sum, are compared at that level: a 1-ulp shift
    of a cut node next to a knot moves
    B ~ (x - xi)^p by many ulps, and minimum-norm weights carry solver-dependent
    noise on entries that are mathematically zero. Entries with S_ij == 0 must
    be exactly zero on the device too. With ``ts`` the five worst entries
    (slot, row, row class, values) are printed.
    """
    m = S > 0
    bad0 = np.nonzero((~m) & (gpu != 0.0))
    assert bad0[0].size == 0, f"{label}: entries with no quadrature terms must be zero: {list(zip(*bad0))[:5]}"
    if not m.any():
        return 0.0
    den = np.maximum(np.maximum(S, floor * np.abs(ref).max()), rowfloor * S.max(axis=0, keepdims=True))
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.where(m, np.abs(gpu - ref) / den, 0.0)
    if ts is not None:
        W = int(round(np.sqrt(ref.shape[0])))
        p = (W - 1) // 2
        for f in np.argsort(rel.ravel())[::-1][:5]:
            s, r = divmod(int(f), ref.shape[1])
            flat = int(ts.active[r])
            say(f"   {label} worst: slot {s} (a={s // W - p}, b={s % W - p}) row {r} (i1={flat % ts.n1}, "
                f"i2={flat // ts.n1}, class {int(ts.fcls.reshape(-1)[flat])}) gpu {gpu[s, r]:.17e} ref {ref[s, r]:.17e} "
                f"S {S[s, r]:.3e} rel {rel[s, r]:.3e}")
    return float(rel.max())


def p3_bound(o):
    """Tolerance of the end-to-end comparison: two backward-stable minimum-norm
    solvers of Eq. (5) agree to about cond(A_i) eps relative, and cut nodes
    computed on each side differ by a few ulps; 1e-10 floor."""
    from oracle import wq
    kappa = max(wq.wq_condition(o.k1, o.p).max(), wq.wq_condition(o.k2, o.p).max())
    return max(1e-10, 1e-15 * kappa), kappa


def oracle_cut_nodes(o):
    """Cut-element nodes of the oracle in the library's order (cut elements in flat order)."""
    xs, ys, ws = [], [], []
    for (e1, e2) in o.ts.cut_elements():
        x, y, w, _ = o.ts.cut_rule(e1, e2)
        xs.append(x)
        ys.append(y)
        ws.append(w)
    if not xs:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


def oracle_weight_table(o, d, qmax):
    """Oracle weights in the library's table layout: row i, column q = point k0(i) + q."""
    W, el = (o.W1, o.el1) if d == 0 else (o.W2, o.el2)
    p = o.p
    n = W.shape[0]
    tab = np.zeros((n, qmax))
    for i in range(n):
        sel = np.nonzero((el >= max(0, i - p)) & (el <= i))[0]
        tab[i, :len(sel)] = W[i, sel]
    return tab


def worst_entries(gpu, ref, ts, k=5):
    """Largest floor-relative deviations with the row class, for failure messages."""
    rowmax = np.abs(ref).max(axis=0, keepdims=True)
    den = np.maximum(np.maximum(np.abs(ref), 1e-3 * rowmax), 1e-300)
    rel = np.abs(gpu - ref) / den
    idx = np.argsort(rel.ravel())[::-1][:k]
    out = []
    for f in idx:
        s, r = divmod(int(f), ref.shape[1])
        flat = ts.active[r]
        out.append(dict(slot=s, row=r, cls=int(ts.fcls.reshape(-1)[flat]), gpu=gpu[s, r], ref=ref[s, r],
                        rel=rel[s, r], rowmax=rowmax[0, r]))
    return out


def oracle_dwq_tables(o, d, KQ):
    """The oracle's discontinuous rules of direction d in the device layout.

    Per slot 2(s-1)+side: the points of the side's first p+1 elements (all
    non-zero weights of the p functions containing t lie there), their
    elements and WQ indices, and the weights of B_{s+ii}, ii = 0..p-1.
    """
    from oracle import dwq
    D = o.dwq_dirs()[d]
    p = o.p
    slots = 2 * (D.N - 1)
    npts = np.zeros(slots, dtype=np.int64)
    X = np.zeros((slots, KQ))
    E = np.full((slots, KQ), -1, dtype=np.int64)
    K = np.full((slots, KQ), -1, dtype=np.int64)
    Wt = np.zeros((slots, p, KQ))
    cond = np.ones(slots)
    for s in range(1, D.N):
        for side in (dwq.LOW, dwq.HIGH):
            sl = 2 * (s - 1) + side
            x, el, k, _, _, _ = D.side_rule(s, side)
            keep = (el <= s + p) if side == dwq.HIGH else (el >= s - 1 - p)
            n = int(keep.sum())
            npts[sl] = n
            X[sl, :n] = x[keep]
            E[sl, :n] = el[keep]
            K[sl, :n] = k[keep]
            for ii in range(p):
                Wt[sl, ii, :n] = D.dwq_weights(s + ii, s, side)[3][keep]
            cond[sl] = D.side_condition(s, side)
    return npts, X, E, K, Wt, cond


def inject_oracle_dwq(plan, o):
    """Give a DWQ plan the oracle's discontinuous weights of both directions (points are identical)."""
    import torch
    from paper_2101_08053_amd import igatrim
    for d in range(2):
        KQ = plan.table(igatrim.TABLE_DWQ_X, d).shape[1]
        *_, Wt, _ = oracle_dwq_tables(o, d, KQ)
        plan.set_dwq_weights(d, torch.as_tensor(np.ascontiguousarray(Wt.reshape(-1, KQ)), device="cuda"))
