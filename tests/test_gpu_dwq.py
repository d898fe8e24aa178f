"""GPU parity of discontinuous weighted quadrature (Sect. 3.3) against the oracle.

* Side tables: point lists (coordinates, elements, WQ indices) match exactly
  up to the last bit of the coordinates (1e-15); the discontinuous weights,
  solved independently (Householder on the device, SVD least squares in the
  oracle), agree row-relatively to max(1e-13, 1e-15 cond), cond being the
  largest condition number of the slot's refined systems.
* Boxes (the choice of region R among the support's inside boxes): identical integers for every row formed element-wise.
* P2 (identical rules: the oracle's WQ weights, discontinuous weights and cut
  nodes injected): <= 1e-12 in the metric of the hybrid tests.
* P3 (the device's own rules): the hybrid bound and floors.
* Table 1, middle column: at c = 1 the DWQ matrix equals element Gauss at
  round-off; the area invariant holds to 1e-10.
"""
import numpy as np
import pytest

from gpu_common import (FLOOR_P3, ROWFLOOR_P3, inject_oracle_dwq, inject_oracle_rules, oracle_dwq_tables, p3_bound,
                        parity_S, require_gpu, say)
from oracle.assemble import Oracle, to_ell
from oracle.geometry import Coefficient
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = {
    "line_p3_N10": lambda: wl.table1_line(3),
    "circle_p2_N40": lambda: wl.config1(N=40),
    "cubic16_p4_N48": lambda: wl.config2(N=48),
    "ellipses3_p6_N30": lambda: wl.config3(N=30),
    "ellipses3_p5_N30": lambda: wl.config3(N=30, p=5),
    "line_p7_N10": lambda: wl.table1_line(7),
    "line_p8_N10": lambda: wl.table1_line(8),
    "circle_p3_N30_nonuniform": lambda: wl.nonuniform_variant(wl.config1(N=30, p=3)),
    "ellipses3_p5_N24_nonuniform": lambda: wl.nonuniform_variant(wl.config3(N=24, p=5)),
}
_oracles = {}


def _oracle(name):
    if name not in _oracles:
        cfg = CASES[name]()
        _oracles[name] = (cfg, Oracle(cfg))
    return _oracles[name]


def _plan(cfg):
    from paper_2101_08053_amd import igatrim
    return igatrim.Plan(cfg, igatrim.DWQ)


@pytest.mark.parametrize("name", list(CASES))
def test_side_tables_match_oracle(name):
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg, o = _oracle(name)
    plan = _plan(cfg)
    plan.status()
    p = cfg.p
    for d in range(2):
        X = plan.table(igatrim.TABLE_DWQ_X, d).cpu().numpy()
        KQ = X.shape[1]
        Wg = plan.table(igatrim.TABLE_DWQ_W, d).cpu().numpy().reshape(-1, p, KQ)
        n = plan.int_table(igatrim.ITABLE_DWQ_NPTS, d).cpu().numpy().ravel()
        E = plan.int_table(igatrim.ITABLE_DWQ_ELEM, d).cpu().numpy()
        K = plan.int_table(igatrim.ITABLE_DWQ_WQIDX, d).cpu().numpy()
        on, oX, oE, oK, oW, cond = oracle_dwq_tables(o, d, KQ)
        np.testing.assert_array_equal(n, on)
        for sl in range(len(n)):
            m = n[sl]
            np.testing.assert_allclose(X[sl, :m], oX[sl, :m], rtol=0, atol=1e-15)
            np.testing.assert_array_equal(E[sl, :m], oE[sl, :m])
            np.testing.assert_array_equal(K[sl, :m], oK[sl, :m])
        scale = np.abs(oW).max(axis=2)
        rel = np.abs(Wg - oW).max(axis=2) / np.where(scale > 0, scale, 1.0)
        tol = np.maximum(1e-13, 1e-15 * cond)[:, None]
        worst = np.unravel_index(np.argmax(rel / tol), rel.shape)
        say(f"[dwq sides] {name} dir {d}: max row-relative weight difference {rel.max():.3e} "
            f"(slot {worst[0]}, cond {cond[worst[0]]:.2e})")
        assert np.all(rel <= tol)


@pytest.mark.parametrize("name", list(CASES))
def test_boxes_match_oracle(name):
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg, o = _oracle(name)
    plan = _plan(cfg)
    rows = plan.int_table(igatrim.ITABLE_FORM_ROWS).cpu().numpy().ravel()
    box = plan.int_table(igatrim.ITABLE_DWQ_BOX).cpu().numpy()
    ts = o.ts
    n_box = 0
    for r, b in zip(rows, box):
        f = int(ts.active[r])
        i2, i1 = divmod(f, ts.n1)
        reg = o.dwq_region(i1, i2)
        if reg is None:
            assert b[0] == -1, (i1, i2, b)
        else:
            assert tuple(b) == tuple(reg[0]) + tuple(reg[1]), (i1, i2, b, reg)
            n_box += 1
    assert plan.sizes["n_dwq_rows"] == n_box
    say(f"[dwq boxes] {name}: {n_box} of {len(rows)} cut rows use a box")


@pytest.mark.parametrize("name", list(CASES))
def test_dwq_parity(name):
    require_gpu()
    cfg, o = _oracle(name)
    say(f"[dwq] {name}")
    plan = _plan(cfg)
    ref = to_ell(o.dwq(), o.ts)
    S = to_ell(o.dwq(absolute=True), o.ts)
    inject_oracle_rules(plan, o)
    inject_oracle_dwq(plan, o)
    v2 = plan.mass_form().cpu().numpy()
    plan.status()
    m2 = parity_S(v2, ref, S, o.ts, "P2")
    say(f"   P2 parity {m2:.3e}")
    assert m2 <= 1e-12
    v3 = plan.mass_form(full=True).cpu().numpy()
    m3 = parity_S(v3, ref, S, o.ts, "P3", FLOOR_P3, ROWFLOOR_P3)
    tol, kappa = p3_bound(o)
    say(f"   P3 parity {m3:.3e} (bound {tol:.1e}, max cond {kappa:.2e})")
    assert m3 <= tol
    assert np.array_equal(v3, plan.mass_form(full=True).cpu().numpy())


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_table1_dwq(p):
    """c = 1 on the line trim: DWQ at round-off from element Gauss (Table 1, middle column)."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.table1_line(p)
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_CONST))
    G = to_ell(o.gauss_reference(), o.ts)
    plan = _plan(cfg)
    v = plan.mass_form(plan.coeff(igatrim.COEF_CONST, 1.0)).cpu().numpy()
    err = np.linalg.norm(v - G)
    say(f"[table1 dwq] p={p}: ||M_dwq - M_gauss||_F = {err:.3e}")
    assert err < 1e-14
    assert abs(v.sum() - o.ts.visible_area()) < 1e-10


def test_dwq_rejects_points_coefficient():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.config1(N=16)
    plan = _plan(cfg)
    ones = torch.ones(plan.sizes["n_points"], dtype=torch.float64, device="cuda")
    c = plan.coeff(igatrim.COEF_AT_POINTS, c_points=ones)
    with pytest.raises(igatrim.IgaError):
        plan.mass_form(c)
