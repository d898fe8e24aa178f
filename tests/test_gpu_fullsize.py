"""GPU parity at the benchmark workloads' full sizes, in the launch configuration bench.py times.

* 256 x 256, p = 4, perturbed geometry (c = |det J|), 16-point cubic hole,
  hybrid Gauss and DWQ; 512 x 512, p = 6, three ellipses, DWQ. The device
  forms the whole matrix (full formation from the raw inputs, replayed as a
  graph); the oracle is set up on the whole patch and computes a seeded
  sample of rows -- interior rows by its own weighted quadrature, cut rows by
  element Gauss with its cut rule (hybrid) or by its DWQ rows. The sampled
  rows must meet the end-to-end bar of the smaller parity tests (P3: the
  device's own weights and nodes, relative to each entry's sum of absolute
  terms, tolerance max(1e-10, 1e-15 max cond)); the compact maps must match
  exactly.
* 1024 x 1024 (the matrix-free workload): y = M(c) u and its adjoint against
  the device's formed matrix at that size (itself checked against the oracle
  at the sizes above), entry by entry relative to the sum of absolute terms
  (1e-12), and <dc, c> = <r, y>, an identity of the adjoint.
* 256 patches of the batched workload: the batched launches equal the
  one-patch formation bit for bit.
* 300 x 300, p = 2, circular hole (c = 1): the cut rules find their elements
  from more class counts than one batch of loads covers; sampled rows as above.
* 256 x 256, p = 4, cubic hole, with a separable map (c = f'(x) g'(y)): sampled
  interior rows equal products of 1-D weighted sums evaluated by SciPy, a
  property that holds at any size and needs no oracle set-up.
"""
import numpy as np
import pytest

from gpu_common import FLOOR_P3, ROWFLOOR_P3, p3_bound, parity_S, require_gpu, say
from oracle.assemble import Oracle, to_ell
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _device_full(plan, igatrim):
    coef = plan.coeff()
    torch = require_gpu()
    out = torch.empty((plan.sizes["band"], plan.sizes["n_act"]), dtype=torch.float64, device="cuda")
    for _ in range(3):  # kernel by kernel, recorded, replayed
        plan.mass_form(coef, out=out, full=True)
    plan.status()
    return out.cpu().numpy()


def _sample(o, n_int, n_cut, seed):
    rng = np.random.default_rng(seed)
    inter, cut = o.interior_rows_flat(), o.cut_rows_flat()
    ri = np.sort(rng.choice(inter, min(n_int, len(inter)), replace=False))
    rc = np.sort(rng.choice(cut, min(n_cut, len(cut)), replace=False))
    return ri, rc


def _support_elements(o, rows):
    p, ts = o.p, o.ts
    els = set()
    for f in rows:
        i2, i1 = divmod(int(f), ts.n1)
        for e2 in range(max(0, i2 - p), min(ts.N2 - 1, i2) + 1):
            for e1 in range(max(0, i1 - p), min(ts.N1 - 1, i1) + 1):
                if ts.ecls[e2, e1] != 0:
                    els.add((e1, e2))
    return sorted(els, key=lambda t: (t[1], t[0]))


def _dwq_into(o, rows, ref, absolute):
    """Oracle DWQ rows (dicts of flat column -> value) into the band layout; rows without a box
    fall back to the hybrid rule, returned for the caller."""
    ts, p = o.ts, o.p
    W = 2 * p + 1
    fallback = []
    for f in rows:
        i2, i1 = divmod(int(f), ts.n1)
        row = o.dwq_row(i1, i2, absolute)
        if row is None:
            fallback.append(f)
            continue
        r = ts.act_of[f]
        for col, v in row.items():
            if ts.act_of[col] < 0:
                continue
            j2, j1 = divmod(col, ts.n1)
            ref[(j1 - i1 + p) * W + (j2 - i2 + p), r] += v
    return np.array(fallback, dtype=np.int64)


def _check_sampled(igatrim, cfg, method, n_int, n_cut, seed):
    say(f"[full size] {cfg.name} method {method}: oracle set-up on the whole patch")
    o = Oracle(cfg)
    ts = o.ts
    plan = igatrim.Plan(cfg, method)
    s = plan.sizes
    act_of, fn_of, fcls = (t.cpu().numpy() for t in plan.index_maps())
    assert s["n_act"] == ts.n_act
    np.testing.assert_array_equal(fcls, ts.fcls.reshape(-1))
    np.testing.assert_array_equal(act_of, ts.act_of)
    say(f"   device formation: n_act {s['n_act']}, cut rows {s['n_cut_fn']}, cut elements {s['n_cut_el']}")
    vals = _device_full(plan, igatrim)
    ri, rc = _sample(o, n_int, n_cut, seed)
    say(f"   oracle rows: {len(ri)} interior, {len(rc)} cut")
    ref = to_ell(o.wq_rows(ri), ts)
    S = to_ell(o.wq_rows(ri, absolute=True), ts)
    if method == igatrim.DWQ:
        fb = _dwq_into(o, rc, ref, False)
        _dwq_into(o, rc, S, True)
        say(f"   {len(rc) - len(fb)} cut rows by DWQ boxes, {len(fb)} by the hybrid rule")
    else:
        fb = rc
    if len(fb):
        els = _support_elements(o, fb)
        ref += to_ell(o.gauss_reference(fb, els), ts)
        S += to_ell(o.gauss_reference(fb, els, absolute=True), ts)
    cols = ts.act_of[np.concatenate([ri, rc])]
    m = parity_S(vals[:, cols], ref[:, cols], S[:, cols], None, "P3", FLOOR_P3, ROWFLOOR_P3)
    tol, kappa = p3_bound(o)
    say(f"   sampled rows: parity {m:.3e} (bound {tol:.1e}, max cond {kappa:.2e})")
    assert m <= tol


def test_fullsize_headline_hybrid():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    _check_sampled(igatrim, wl.config2(), igatrim.HYBRID_GAUSS, 300, 120, 11)


def test_fullsize_headline_dwq():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    _check_sampled(igatrim, wl.config2(), igatrim.DWQ, 150, 60, 12)


def test_fullsize_high_degree_dwq():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    _check_sampled(igatrim, wl.config3(), igatrim.DWQ, 100, 30, 13)


def test_fullsize_cut_rules_locate_past_one_batch():
    """300 x 300, p = 2, circular hole: 300 element rows of 19 tile columns, so each cut-rule
    workgroup sums the class kernel's counts in two batches of loads before finding its element
    (the headline's 256 x 16 counts take one); sampled rows against the oracle."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    _check_sampled(igatrim, wl.config1(N=300, p=2), igatrim.HYBRID_GAUSS, 100, 150, 14)


def test_fullsize_matrix_free():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.config5()
    say(f"[full size] {cfg.name}: matrix-free product and adjoint against the formed matrix")
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    s = plan.sizes
    pts = plan.points()
    c = wl.config5_coef(pts[:, 0], pts[:, 1], torch).contiguous()
    u_np, f_np = wl.config5_vectors(s["n_act"])
    u = torch.as_tensor(u_np, device="cuda")
    gy = torch.as_tensor(f_np, device="cuda")
    y = igatrim.mf_apply(plan, c, u)
    du, dc = igatrim.mf_adjoint(plan, c, u, gy)
    coef = plan.coeff(igatrim.COEF_AT_POINTS, c_points=c)
    vals = torch.empty((s["band"], s["n_act"]), dtype=torch.float64, device="cuda")
    for _ in range(3):
        plan.mass_form(coef, out=vals)
    plan.status()
    act_of, fn_of, _ = plan.index_maps()
    act_of, fn_of = act_of.long(), fn_of.long()
    p, n1, n2 = s["p"], s["n1"], s["n2"]
    W = 2 * p + 1
    i1, i2 = fn_of % n1, fn_of // n1
    y_ref = torch.zeros_like(u)
    y_abs = torch.zeros_like(u)
    du_ref = torch.zeros_like(u)
    du_abs = torch.zeros_like(u)
    for sl in range(W * W):
        a, b = sl // W - p, sl % W - p
        j1, j2 = i1 + a, i2 + b
        ok = (j1 >= 0) & (j1 < n1) & (j2 >= 0) & (j2 < n2)
        cid = torch.where(ok, act_of[(j2.clamp(0, n2 - 1) * n1 + j1.clamp(0, n1 - 1))], torch.full_like(j1, -1))
        live = cid >= 0
        m = torch.where(live, vals[sl], torch.zeros_like(vals[sl]))
        cc = cid.clamp(min=0)
        y_ref += m * u[cc]
        y_abs += m.abs() * u[cc].abs()
        du_ref.index_add_(0, cc, m * gy)
        du_abs.index_add_(0, cc, m.abs() * gy.abs())
    ey = ((y - y_ref).abs() / y_abs.clamp(min=1e-300)).max().item()
    edu = ((du - du_ref).abs() / du_abs.clamp(min=1e-300)).max().item()
    lhs, rhs = (dc * c).sum().item(), (gy * y).sum().item()
    eid = abs(lhs - rhs) / (dc * c).abs().sum().item()
    say(f"   y: {ey:.2e}, du: {edu:.2e}, <dc, c> - <r, y>: {eid:.2e} (n_act {s['n_act']}, points {s['n_points']})")
    assert ey <= 1e-12 and edu <= 1e-12 and eid <= 1e-12


def test_fullsize_batched():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs = wl.config4()
    say(f"[full size] batched workload: {len(cfgs)} patches")
    plans = [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]
    coeffs = [p.coeff() for p in plans]
    ref = [p.mass_form(c).cpu().numpy() for p, c in zip(plans, coeffs)]
    b = igatrim.Batch(plans, coeffs)
    b.autotune()
    for o in b.outs:
        o.fill_(np.nan)
    outs = [o.cpu().numpy() for o in b.form(use_graph=True)]
    b.status()
    bad = [k for k, (g, r) in enumerate(zip(outs, ref)) if not np.array_equal(g, r)]
    say(f"   {len(cfgs) - len(bad)} of {len(cfgs)} patches bit-identical; info {b.info()}")
    assert not bad


def test_fullsize_separable_map_rows_factorise():
    """256 x 256, p = 4, cubic hole, graph replay: interior rows with a non-constant c against a property.

    With a separable map F(x, y) = (f(x), g(y)), c = |det J| = f'(x) g'(y), and
    an interior row's entry for column (j1, j2) is the product of the 1-D sums
    sum_k w1_{k,i1} f'(x_k) B_j1(x_k) and sum_l w2_{l,i2} g'(y_l) B_j2(y_l)
    (Eq. (7) with a separable c). The device's own weights and points, SciPy's
    f', g' and basis values give the products; 400 sampled interior rows of
    the device's full formation must match them to 1e-12 of the row's largest
    entry (the device sums the same terms in another order).
    """
    torch = require_gpu()
    from scipy.interpolate import BSpline
    from paper_2101_08053_amd import igatrim
    p, N = 4, 256
    cfg = wl.config2(N=N, p=p)
    g1, g2 = wl.greville(cfg.knots[0], p), wl.greville(cfg.knots[1], p)
    a, b = g1 + 0.2 * g1 ** 2, g2 - 0.15 * g2 ** 2   # increasing: f', g' > 0
    cp = np.empty((len(g2), len(g1), 2))
    cp[..., 0] = a[None, :]
    cp[..., 1] = b[:, None]
    cfg.geom_cp = cp
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    vals = _device_full(plan, igatrim)
    act_of, _, fcls = (t.cpu().numpy() for t in plan.index_maps())
    n1, W = plan.sizes["n1"], 2 * p + 1

    def pt0(e, Ne):  # first WQ point of element e: p+1 points in the end elements, 2 in the others
        return 0 if e <= 0 else (p + 1) + 2 * (e - 1)

    factors = []
    for d, coefs in ((0, a), (1, b)):
        xq = plan.table(igatrim.TABLE_WQ_POINTS, d).cpu().numpy().ravel()
        Wt = plan.table(igatrim.TABLE_WQ_WEIGHTS, d).cpu().numpy()
        knots = cfg.knots[d]
        fp = BSpline(knots, coefs, p).derivative()(xq)
        B = BSpline.design_matrix(xq, knots, p).toarray()
        Wfull = np.zeros((Wt.shape[0], len(xq)))
        for i in range(Wt.shape[0]):
            k0 = pt0(max(0, i - p), N)
            q = min(Wt.shape[1], len(xq) - k0)
            Wfull[i, k0:k0 + q] = Wt[i, :q]
        factors.append((Wfull * fp[None, :]) @ B)   # [i, j]
    F1, F2 = factors
    interior = np.nonzero(fcls == 1)[0]   # function class 1: interior
    rows = np.sort(np.random.default_rng(wl.SEED_BASE + 77).choice(interior, 400, replace=False))
    worst = 0.0
    for f in rows:
        i2, i1 = divmod(int(f), n1)
        r = act_of[f]
        got = np.zeros((W, W))
        exp = np.zeros((W, W))
        for ai in range(W):
            for bi in range(W):
                j1, j2 = i1 + ai - p, i2 + bi - p
                if 0 <= j1 < n1 and 0 <= j2 < plan.sizes["n2"] and act_of[j2 * n1 + j1] >= 0:
                    got[ai, bi] = vals[ai * W + bi, r]
                    exp[ai, bi] = F1[i1, j1] * F2[i2, j2]
        worst = max(worst, np.abs(got - exp).max() / np.abs(exp).max())
    say(f"[separable map 256^2 p4] {len(rows)} interior rows: max |device - product| / row max = {worst:.2e}")
    assert worst <= 1e-12
