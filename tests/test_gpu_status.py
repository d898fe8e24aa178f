"""Error returns of the C ABI: every failure is an ordinary status code.

Each case reaches its code through valid calls (no kernel is made to fault):
argument and knot checks on the host, a weight system of Eq. (5) that is
inconsistent for a legal but degenerate knot vector (the oracle's own
least-squares residual confirms it), a trimming polygon that crosses one
element edge more often than a cut rule holds, and a PCG capped at one
iteration. The device-side codes come back through the plan's status word.
"""
import ctypes as C
import math

import numpy as np
import pytest

from gpu_common import require_gpu, say
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _code(fn, *a, **kw):
    from paper_2101_08053_amd import igatrim
    try:
        fn(*a, **kw)
    except igatrim.IgaError as e:
        return e.code
    return 0


def _plan(cfg, method=None, **kw):
    from paper_2101_08053_amd import igatrim
    return igatrim.Plan(cfg, igatrim.HYBRID_GAUSS if method is None else method, **kw)


def test_invalid_knots():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    p, N = 2, 8
    good = wl.open_uniform_knots(N, p)
    bad = {
        "not open at 0": np.concatenate([[0.0, 0.0, 0.05], good[3:]]),
        "not open at 1": np.concatenate([good[:-3], [0.95, 1.0, 1.0]]),
        "decreasing": np.concatenate([good[:5], [good[4] - 0.01], good[6:]]),
        "repeated interior": np.concatenate([good[:5], [good[4]], good[6:]]),
        "too short": np.array([0.0, 0.0, 1.0, 1.0]),
    }
    for name, k in bad.items():
        cfg = wl.Patch(p=p, n_el=(N, N), knots=(k, good), curves=[wl.circle(0.5, 0.5, 0.25)])
        code = _code(_plan, cfg)
        say(f"[status] {name}: {igatrim.STATUS.get(code, code)}")
        assert code == -1, name


def test_unsupported_inputs():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    for p in (0, 9):
        k = wl.open_uniform_knots(6, max(p, 1))
        cfg = wl.Patch(p=p, n_el=(6, 6), knots=(k, k))
        assert _code(_plan, cfg) == -2, p
    cfg = wl.config1(N=8)
    cfg.curves = [wl.Curve(kind=wl.CURVE_BSPLINE, degree=4, cp=np.random.default_rng(0).random((8, 2)))]
    assert _code(_plan, cfg) == -2
    cfg = wl.config2(N=8, p=2)
    cfg.curves = cfg.curves * 2  # several holes are handled for ellipses only
    assert _code(_plan, cfg) == -2
    assert _code(_plan, wl.config1(N=8), method=7) == -2
    plan = _plan(wl.config1(N=8), igatrim.DWQ)
    ones = torch.ones(plan.sizes["n_points"], dtype=torch.float64, device="cuda")
    assert _code(plan.mass_form, plan.coeff(igatrim.COEF_AT_POINTS, c_points=ones)) == -2


def test_invalid_arguments():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    L = igatrim.lib()
    cfg = wl.config1(N=8)
    plan = _plan(cfg)
    # reserved option fields
    desc_plan = C.c_void_p()
    assert L.iga_trim_plan_create(None, None, C.byref(desc_plan)) == -1
    # a cut-node injection with the wrong count
    n = plan.sizes["n_cut_nodes"]
    x = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    assert _code(plan.set_cut_nodes, x, x, x) == -1
    # DWQ weights into a plan of another method
    assert _code(plan.set_dwq_weights, 0, x) == -1
    # directions other than 0 and 1
    assert _code(plan.table, igatrim.TABLE_WQ_POINTS, 2) == -1
    # rtol and maxit must be positive
    c = plan.coeff(igatrim.COEF_CONST, 1.0)
    vals = plan.mass_form(c)
    g = igatrim.target_sincos(math.pi, 0.0, math.pi, 0.0)
    assert _code(igatrim.l2_project, plan, vals, c, g, rtol=0.0) == -1


def test_reserved_option_fields_rejected():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.config1(N=8)
    desc = igatrim.iga_patch_desc()
    desc.degree, desc.method = cfg.p, igatrim.HYBRID_GAUSS
    keep = []
    for d in range(2):
        k = np.ascontiguousarray(cfg.knots[d])
        keep.append(k)
        desc.n_knots[d] = len(k)
        desc.knots[d] = k.ctypes.data_as(C.POINTER(C.c_double))
    opts = igatrim.iga_opts()
    opts.reserved[2] = 64
    h = C.c_void_p()
    assert igatrim.lib().iga_trim_plan_create(C.byref(desc), C.byref(opts), C.byref(h)) == -1
    opts.reserved[2] = 0
    assert igatrim.lib().iga_trim_plan_create(C.byref(desc), C.byref(opts), C.byref(h)) == 0
    igatrim.lib().iga_plan_destroy(h)


def test_singular_weight_system():
    """Three consecutive elements one ulp wide (p = 3): the minimum-norm system of Eq. (5) of a
    function supported there has no solution; the device's residual check reports it."""
    require_gpu()
    from oracle import wq
    p = 3
    t = 0.5
    a = np.nextafter(t, 1.0)
    b = np.nextafter(a, 1.0)
    c = np.nextafter(b, 1.0)
    k = np.array([0.0] * 4 + [0.25, t, a, b, c, 0.75] + [1.0] * 4)
    xs, el = wq.wq_points(k, p)
    _, res = wq.wq_weights(k, p, xs, el, wq.mass_1d(k, p), True)
    say(f"[status] oracle residual of Eq. (5) on the degenerate knots: {np.max(res):.2e}")
    assert np.max(res) > 1e-6  # the oracle finds the same system inconsistent
    good = wl.open_uniform_knots(6, p)
    cfg = wl.Patch(p=p, n_el=(len(k) - 2 * p - 1, 6), knots=(k, good))
    assert _code(_plan, cfg) == -5
    # the uniform patch of the same degree is fine
    assert _code(_plan, wl.Patch(p=p, n_el=(6, 6), knots=(good, good))) == 0


def _zigzag(n_teeth=20):
    """A hole polygon that crosses the grid line x = 1/4 of a 4 x 4 patch n_teeth + 1 times inside
    one element row (more split points than one element edge of a cut rule holds)."""
    pts = [(0.2 if k % 2 == 0 else 0.3, 0.27 + 0.01 * k) for k in range(n_teeth)]
    pts += [(0.6, pts[-1][1]), (0.6, 0.26), (0.3, 0.26)]
    return wl.Curve(kind=wl.CURVE_BSPLINE, degree=1, cp=np.array(pts))


def test_topology_overflow():
    require_gpu()
    p, N = 2, 4
    k = wl.open_uniform_knots(N, p)
    cfg = wl.Patch(p=p, n_el=(N, N), knots=(k, k), curves=[_zigzag()])
    assert _code(_plan, cfg) == -6
    # a few teeth stay within the rule's capacity
    cfg.curves = [_zigzag(4)]
    assert _code(_plan, cfg) == 0


def test_no_convergence_returns_last_iterate():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    plan = _plan(wl.config1(N=16))
    c = plan.coeff(igatrim.COEF_CONST, 1.0)
    vals = plan.mass_form(c)
    g = igatrim.target_sincos(math.pi, 0.0, math.pi, 0.0)
    u, info = igatrim.l2_project(plan, vals, c, g, rtol=1e-12, maxit=1, raise_on_noconv=False)
    say(f"[status] maxit = 1: {info}")
    assert info["iterations"] == 1 and not info["converged"]
    assert math.isfinite(info["rel_residual"]) and info["rel_residual"] > 1e-12
    assert bool(torch.isfinite(u).all())
    assert _code(igatrim.l2_project, plan, vals, c, g, rtol=1e-12, maxit=1) == -8


def test_pcg_past_convergence_stays_finite():
    """Iterations after the residual has vanished take zero steps (no 0/0): on a 9-function
    untrimmed patch, 300 iterations towards an unreachable tolerance leave the converged solution."""
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    k = wl.open_uniform_knots(2, 1)
    plan = _plan(wl.Patch(p=1, n_el=(2, 2), knots=(k, k)))
    c = plan.coeff(igatrim.COEF_CONST, 1.0)
    vals = plan.mass_form(c)
    g = igatrim.target_sincos(2.0, 0.0, 3.0, 0.0)
    u_ok, info_ok = igatrim.l2_project(plan, vals, c, g, rtol=1e-13)
    u, info = igatrim.l2_project(plan, vals, c, g, rtol=1e-300, maxit=300, raise_on_noconv=False)
    say(f"[status] 300 iterations on 9 functions: {info}")
    # a residual of exactly zero counts as converged; otherwise all 300 iterations ran
    assert (info["iterations"] == 300) or (info["converged"] and info["rel_residual"] == 0.0)
    assert bool(torch.isfinite(u).all())
    assert float((u - u_ok).abs().max()) <= 1e-12 * float(u_ok.abs().max())
