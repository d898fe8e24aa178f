"""GPU parity of mass formation (Eq. (6) over the visible domain) against the oracle.

Metric: max |dM_ij| / S_ij with S_ij = sum of |w c B_i B_j| over the entry's
quadrature terms (the entry's relative error measured against the scale of its
own rounding; it equals the plain relative error when no term cancels).
* P1 -- weights of Eq. (5), solved independently on each side (Householder QR
  of A^T on the device, SVD least squares in the oracle): row-relative
  difference <= max(1e-13, 1e-15 cond(A_i)).
* P2 -- formation under identical rules (the oracle's weights and cut nodes
  injected): <= 1e-12, no floor.
* P3 -- end to end with the device's own weights and nodes: <= max(1e-10,
  1e-15 max_i cond(A_i)), entries floored at 1e-3 of their row's largest term
  sum and 1e-5 of the largest entry; for p = 6 the systems next to the patch
  boundary reach cond ~ 1e7, and two NumPy solvers already differ by ~3e-10
  there. The global floor is 1e-5 because minimum-norm weights from two
  different solvers leave noise of ~1e-18 on entries that are mathematically
  zero (naive WQ rows cut by the line trim measured 2.6e-7 relative at a
  1e-9 floor); the identical-rule comparison (P2) has no floor at all.
Integer data (classes, compaction maps, counts) match exactly.
"""
import math

import numpy as np
import pytest

from gpu_common import (FLOOR_P3, ROWFLOOR_P3, inject_oracle_rules, oracle_cut_nodes, oracle_weight_table, p3_bound,
                        parity_S, require_gpu, say)
from oracle.assemble import Oracle, to_ell
from oracle.geometry import Coefficient
from oracle.trim import CUT_FN, EXTERIOR_FN
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = {
    "circle_p2_N100": lambda: wl.config1(N=100),
    "cubic16_p4_N80": lambda: wl.config2(N=80),
    "ellipses3_p6_N70": lambda: wl.config3(N=70),
    "ellipses3_p3_N40": lambda: wl.config3(N=40, p=3),
    "line_p3_N10": lambda: wl.table1_line(3),
    "circle_p2_N70": lambda: wl.config1(N=70),
    "circle_p7_N24": lambda: wl.config1(N=24, p=7),
    "cubic16_p8_N20": lambda: wl.config2(N=20, p=8),
    # non-uniform simple knots (interior knots jittered by up to 0.3 h)
    "circle_p3_N30_nonuniform": lambda: wl.nonuniform_variant(wl.config1(N=30, p=3)),
    "cubic16_p4_N40_nonuniform": lambda: wl.nonuniform_variant(wl.config2(N=40, p=4)),
}
_oracles = {}


def _oracle(name):
    if name not in _oracles:
        cfg = CASES[name]()
        _oracles[name] = (cfg, Oracle(cfg))
    return _oracles[name]


@pytest.mark.parametrize("name", list(CASES))
def test_structure_matches_oracle(name):
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg, o = _oracle(name)
    say(f"[structure] {name}")
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    s = plan.sizes
    ts = o.ts
    assert s["n_act"] == ts.n_act
    assert s["n_cut_el"] == len(ts.cut_elements())
    act_of, fn_of, fcls = (t.cpu().numpy() for t in plan.index_maps())
    np.testing.assert_array_equal(fcls, ts.fcls.reshape(-1))
    np.testing.assert_array_equal(act_of, ts.act_of)
    np.testing.assert_array_equal(fn_of, ts.active)
    assert s["n_band_el"] == int(ts.band.sum())
    # cut-element nodes, same order and values
    ox, oy, ow = oracle_cut_nodes(o)
    pts = plan.points().cpu().numpy()
    off = s["q1"] * s["q2"] + s["n_band_el"] * (cfg.p + 1) ** 2
    if s["n_cut_nodes"] != len(ow):
        from oracle import bspline
        gx, gy = pts[off:, 0], pts[off:, 1]
        ge = bspline.element_of(ts.bp2, gy) * ts.N1 + bspline.element_of(ts.bp1, gx)
        oe = bspline.element_of(ts.bp2, oy) * ts.N1 + bspline.element_of(ts.bp1, ox)
        gc = np.bincount(ge, minlength=ts.N1 * ts.N2)
        oc = np.bincount(oe, minlength=ts.N1 * ts.N2)
        for e in np.nonzero(gc != oc)[0][:6]:
            e2, e1 = divmod(int(e), ts.N1)
            x, y, w, var = ts.cut_rule(e1, e2)
            say(f"   element ({e1},{e2}): device {gc[e]} nodes, oracle {oc[e]} (variant {var}, arcs "
                f"{[(a[0], a[1], round(a[2], 15), round(a[3], 15)) for a in ts.arcs_of.get((e1, e2), [])]}")
    assert s["n_cut_nodes"] == len(ow)
    np.testing.assert_allclose(pts[off:, 0], ox, rtol=0, atol=1e-13)
    np.testing.assert_allclose(pts[off:, 1], oy, rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", list(CASES))
def test_weight_tables_p1(name):
    """P1: the device's weights of Eq. (5) against the oracle's (independent solvers)."""
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg, o = _oracle(name)
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    from oracle import wq
    for d in range(2):
        Wg = plan.table(igatrim.TABLE_WQ_WEIGHTS, d).cpu().numpy()
        Wo = oracle_weight_table(o, d, Wg.shape[1])
        kappa = wq.wq_condition(cfg.knots[d], cfg.p)
        rel = np.abs(Wg - Wo).max(axis=1) / np.abs(Wo).max(axis=1)
        say(f"[P1] {name} dir {d}: max row-relative weight difference {rel.max():.3e} (row {rel.argmax()}, "
            f"cond {kappa[rel.argmax()]:.2e})")
        assert np.all(rel <= np.maximum(1e-13, 1e-15 * kappa))
        xq = plan.table(igatrim.TABLE_WQ_POINTS, d).cpu().numpy().ravel()
        np.testing.assert_allclose(xq, o.xs1 if d == 0 else o.xs2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", list(CASES))
def test_hybrid_parity(name):
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg, o = _oracle(name)
    say(f"[hybrid] {name}")
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    ref = to_ell(o.hybrid(), o.ts)
    S = to_ell(o.hybrid(absolute=True), o.ts)
    # P2: formation under the oracle's weights and cut nodes
    inject_oracle_rules(plan, o)
    v2 = plan.mass_form().cpu().numpy()
    plan.status()
    m2 = parity_S(v2, ref, S, o.ts, "P2")
    if cfg.coef == wl.COEF_GEOM_DETJ:
        cg = plan.table(igatrim.TABLE_C_WQ).cpu().numpy().reshape(len(o.xs2), len(o.xs1)).T
        co = o.wq_grid_coef()
        say(f"   c on WQ grid: max rel diff {np.abs(cg - co).max() / np.abs(co).max():.3e}")
    say(f"   P2 parity {m2:.3e}")
    assert m2 <= 1e-12
    # P3: end to end with the device's own weights (rebuilt by a full formation)
    v3 = plan.mass_form(full=True).cpu().numpy()
    m3 = parity_S(v3, ref, S, o.ts, "P3", FLOOR_P3, ROWFLOOR_P3)
    tol, kappa = p3_bound(o)
    say(f"   P3 parity {m3:.3e} (bound {tol:.1e}, max cond {kappa:.2e})")
    assert m3 <= tol
    vals2 = plan.mass_form(full=True).cpu().numpy()
    assert np.array_equal(v3, vals2)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_table1_methods(p):
    """Reference Gauss, hybrid and naive WQ on the line trim (Table 1 setting), c = 1."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.table1_line(p)
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_CONST))
    say(f"[table1] p={p}")
    G = to_ell(o.gauss_reference(), o.ts)
    SG = to_ell(o.gauss_reference(absolute=True), o.ts)
    SH = to_ell(o.hybrid(absolute=True), o.ts)
    SN = to_ell(o.naive(absolute=True), o.ts)
    tol, _ = p3_bound(o)
    outs, own = {}, {}
    for meth in (igatrim.GAUSS_REF, igatrim.HYBRID_GAUSS, igatrim.NAIVE_WQ):
        plan = igatrim.Plan(cfg, meth)
        c1 = plan.coeff(igatrim.COEF_CONST, 1.0)
        own[meth] = plan.mass_form(c1).cpu().numpy()
        inject_oracle_rules(plan, o)
        outs[meth] = plan.mass_form(c1).cpu().numpy()
    H, N = to_ell(o.hybrid(), o.ts), to_ell(o.naive(), o.ts)
    assert parity_S(outs[igatrim.GAUSS_REF], G, SG, o.ts, "ref") <= 1e-12
    assert parity_S(outs[igatrim.HYBRID_GAUSS], H, SH, o.ts, "hybrid") <= 1e-12
    assert parity_S(outs[igatrim.NAIVE_WQ], N, SN, o.ts, "naive") <= 1e-12
    assert parity_S(own[igatrim.GAUSS_REF], G, SG, o.ts, "ref own", FLOOR_P3, ROWFLOOR_P3) <= tol
    assert parity_S(own[igatrim.HYBRID_GAUSS], H, SH, o.ts, "hybrid own", FLOOR_P3, ROWFLOOR_P3) <= tol
    assert parity_S(own[igatrim.NAIVE_WQ], N, SN, o.ts, "naive own", FLOOR_P3, ROWFLOOR_P3) <= tol
    outs = own
    # Table 1: hybrid at round-off from the reference, naive WQ far from it
    assert np.linalg.norm(outs[igatrim.HYBRID_GAUSS] - G) < 1e-14
    assert np.linalg.norm(outs[igatrim.NAIVE_WQ] - G) > 1e-5


def test_area_invariant_c1():
    """sum_ij M_ij = visible area (1 - pi/16 for the circle), c = 1."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    for N in (32, 100):
        cfg = wl.config1(N=N)
        plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
        vals = plan.mass_form(plan.coeff(igatrim.COEF_CONST, 1.0)).cpu().numpy()
        assert abs(vals.sum() - (1 - math.pi / 16)) < 1e-10


def test_untrimmed_kronecker():
    require_gpu()
    from oracle import wq
    from paper_2101_08053_amd import igatrim
    p, N1 = 3, 70
    cfg = wl.Patch(p=p, n_el=(N1, 9), knots=(wl.open_uniform_knots(N1, p), wl.open_uniform_knots(9, p)))
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    vals = plan.mass_form(plan.coeff(igatrim.COEF_CONST, 1.0)).cpu().numpy()
    M1, M2 = wq.mass_1d(cfg.knots[0], p), wq.mass_1d(cfg.knots[1], p)
    n1, n2 = N1 + p, 9 + p
    W = 2 * p + 1
    ref = np.zeros_like(vals)
    for s in range(W * W):
        a, b = s // W - p, s % W - p
        for r in range(n1 * n2):
            i1, i2 = r % n1, r // n1
            j1, j2 = i1 + a, i2 + b
            if 0 <= j1 < n1 and 0 <= j2 < n2:
                ref[s, r] = M1[i1, j1] * M2[i2, j2]
    assert np.abs(vals - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("method", ["HYBRID_GAUSS", "DWQ", "GAUSS_REF"])
def test_graph_replay_equals_launches(method):
    """Graph replays of the formation give the kernel-by-kernel result bit for bit.

    Three calls per setting (run kernel by kernel, recorded, replayed) with
    unrelated torch work and synchronisations between them, full and fast
    calls, a new coefficient value (a new recording), and injected weights
    read by a replay.
    """
    require_gpu()
    import torch
    from paper_2101_08053_amd import igatrim
    cfg, o = _oracle("ellipses3_p3_N40")
    m = getattr(igatrim, method)
    say(f"[graph] {method}")
    g = igatrim.Plan(cfg, m)
    g.set_graph(True)
    e = igatrim.Plan(cfg, m)
    e.set_graph(False)
    shape = (g.sizes["band"], g.sizes["n_act"])
    out_g = torch.empty(shape, dtype=torch.float64, device="cuda")
    out_e = torch.empty(shape, dtype=torch.float64, device="cuda")
    for value, full in ((1.0, True), (1.0, True), (1.0, False), (0.75, True), (0.75, False)):
        ref = e.mass_form(e.coeff(igatrim.COEF_CONST, value), out=out_e, full=full).clone()
        for rep in range(3):
            out_g.fill_(float("nan"))
            torch.cuda.synchronize()
            g.mass_form(g.coeff(igatrim.COEF_CONST, value), out=out_g, full=full)
            junk = torch.randn(4096, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            assert torch.equal(out_g, ref), f"replay {rep} (c = {value}, full = {full}) differs"
    g.status()
    if method != "DWQ":
        inject_oracle_rules(g, o)
        inject_oracle_rules(e, o)
        c = igatrim.COEF_CONST
        ref = e.mass_form(e.coeff(c, 0.75), out=out_e, full=False)
        got = g.mass_form(g.coeff(c, 0.75), out=out_g, full=False)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)


def test_points_rewritten_by_full_formation():
    """A full formation rewrites the rule-point table (by the |det J| kernels, or the point kernel
    for other coefficients) with the values plan creation wrote."""
    require_gpu()
    import torch
    from paper_2101_08053_amd import igatrim
    cfg, _ = _oracle("cubic16_p4_N80")
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    p0 = plan.points().clone()
    for coef in (plan.coeff(igatrim.COEF_GEOM_DETJ), plan.coeff(igatrim.COEF_CONST, 1.0)):
        # clobber the table so that only the formation can restore it
        n = p0.numel()
        junk = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        import ctypes as C
        ptr, cnt = C.c_void_p(), C.c_int64()
        igatrim._check(igatrim.lib().iga_plan_points(plan.h, C.byref(ptr), C.byref(cnt)))
        igatrim._check(igatrim.lib().iga_copy(ptr, igatrim._dptr(junk), 8 * n, igatrim._stream()))
        plan.mass_form(coef, full=True)
        torch.cuda.synchronize()
        assert torch.equal(plan.points(), p0)


@pytest.mark.parametrize("N", [100, 400])
def test_lists_are_compactions_of_the_classes(N):
    """Compact maps and lists equal the flat-order compaction of the device's own classes, on a
    patch small enough for each row's workgroup to sum its offset (N = 100) and one large enough
    for the separate offset scan (N = 400)."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.config1(N=N)
    say(f"[lists] N={N}")
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    s = plan.sizes
    act_of, fn_of, fcls = (t.cpu().numpy() for t in plan.index_maps())
    active = fcls != EXTERIOR_FN
    ref_act = np.where(active, np.cumsum(active) - 1, -1)
    np.testing.assert_array_equal(act_of, ref_act)
    np.testing.assert_array_equal(fn_of[: s["n_act"]], np.nonzero(active)[0])
    assert s["n_act"] == int(active.sum())
    assert s["n_cut_fn"] == int((fcls == CUT_FN).sum())
    rows = plan.int_table(igatrim.ITABLE_FORM_ROWS).cpu().numpy().reshape(-1)
    np.testing.assert_array_equal(rows[: s["n_cut_fn"]], ref_act[fcls == CUT_FN])
