"""GPU matrix-free product y = M(c) u and its hand-written adjoint against the oracle.

Tolerances: under identical rules (the oracle's weights and cut nodes
injected) y, du and dc are compared entry by entry against the oracle's
explicit operators What diag(c) Bmat, relative to the sum of absolute terms
of each entry (1e-12); with the device's own rules the same comparison is
made at 1e-9 (the cut nodes differ by ulps, amplified next to knots); the
gradient is also checked by central differences of
the device's own loss (L is quadratic in u and c, so the differences are exact
up to cancellation) on a 16x16-element instance.
"""
import numpy as np
import pytest

from gpu_common import inject_oracle_rules, require_gpu, say
from oracle import matfree
from oracle.assemble import Oracle
from oracle.geometry import Coefficient
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _setup(N, p=4, inject=True):
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.config5(N=N, p=p)
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    o = Oracle(cfg, coef=Coefficient(cfg, kind=wl.COEF_AT_POINTS, field=wl.config5_coef))
    if inject:
        inject_oracle_rules(plan, o)
    pts = plan.points()
    c = wl.config5_coef(pts[:, 0], pts[:, 1], torch).contiguous()
    return torch, igatrim, cfg, plan, c, o


def _close(dev, ref, scale, tol, label):
    err = np.max(np.abs(dev - ref) / np.maximum(scale, 1e-300))
    say(f"   {label}: {err:.2e}")
    assert err <= tol


# one band of elements (N = 16), several bands (72, 40: rows whose support spans two
# bands are summed from both), several strips of test columns (140), degrees 1, 2, 4, 6
# and 8 (32 band elements to a workgroup at degree 1; at degree 8 one, and more reciprocals
# per span than a wavefront has lanes)
@pytest.mark.parametrize("N,p,inject", [(16, 4, True), (72, 4, True), (72, 4, False), (140, 4, True),
                                        (40, 2, True), (40, 6, True), (24, 1, True), (24, 8, True)])
def test_apply_and_adjoint_match_oracle(N, p, inject):
    torch, igatrim, cfg, plan, c, o = _setup(N, p=p, inject=inject)
    tol = 1e-12 if inject else 1e-9
    say(f"[mf] p={p} N={N} n_act={plan.sizes['n_act']} n_points={plan.sizes['n_points']}")
    What, Bmat = matfree.operators(o)
    x, y, *_ = matfree.rule_points(o)
    pts = plan.points().cpu().numpy()
    assert len(x) == len(pts)
    np.testing.assert_allclose(pts[:, 0], x, atol=1e-13, rtol=0)
    np.testing.assert_allclose(pts[:, 1], y, atol=1e-13, rtol=0)
    if not inject:
        x, y = pts[:, 0], pts[:, 1]   # the same field on the device's own points
    cn = wl.config5_coef(x, y)
    u, f = wl.config5_vectors(plan.sizes["n_act"])
    ut = torch.as_tensor(u, device="cuda")
    yd = igatrim.mf_apply(plan, c, ut).cpu().numpy()
    yo = matfree.apply(What, Bmat, cn, u)
    aW, aB = abs(What), abs(Bmat)
    _close(yd, yo, aW @ (np.abs(cn) * (aB @ np.abs(u))), tol, "y")
    gy = np.random.default_rng(2).standard_normal(len(u))
    du, dc = igatrim.mf_adjoint(plan, c, ut, torch.as_tensor(gy, device="cuda"))
    du, dc = du.cpu().numpy(), dc.cpu().numpy()
    R = What.T @ gy
    du_o = Bmat.T @ (cn * R)
    dc_o = (Bmat @ u) * R
    aR = aW.T @ np.abs(gy)
    _close(du, du_o, aB.T @ (np.abs(cn) * aR), tol, "du")
    _close(dc, dc_o, (aB @ np.abs(u)) * aR, tol, "dc")


def test_apply_equals_formed_matrix():
    """M(c) u from the kernels equals the formed band matrix (same c) times u."""
    torch, igatrim, cfg, plan, c, o = _setup(24)
    vals = plan.mass_form(plan.coeff(igatrim.COEF_AT_POINTS, c_points=c)).cpu().numpy()
    from oracle.assemble import from_ell
    M = from_ell(vals, o.ts)
    u = np.random.default_rng(3).standard_normal(plan.sizes["n_act"])
    yd = igatrim.mf_apply(plan, c, torch.as_tensor(u, device="cuda")).cpu().numpy()
    ref = M @ u
    assert np.abs(yd - ref).max() <= 1e-12 * (abs(M) @ np.abs(u)).max()


def test_autograd_and_finite_differences():
    """L = 1/2 ||M(c) u - f||^2 through torch.autograd: oracle gradient and central differences."""
    torch, igatrim, cfg, plan, c, o = _setup(16)
    u, f = wl.config5_vectors(plan.sizes["n_act"])
    ut = torch.as_tensor(u, device="cuda").requires_grad_(True)
    ct = c.clone().requires_grad_(True)
    ft = torch.as_tensor(f, device="cuda")
    yv = igatrim.mass_apply(ut, ct, plan)
    L = 0.5 * ((yv - ft) ** 2).sum()
    L.backward()
    du, dc = ut.grad.cpu().numpy(), ct.grad.cpu().numpy()
    What, Bmat = matfree.operators(o)
    x, y, *_ = matfree.rule_points(o)
    Lo, du_o, dc_o = matfree.gradient(What, Bmat, wl.config5_coef(x, y), u, f)
    assert abs(L.item() - Lo) <= 1e-12 * Lo
    assert np.abs(du - du_o).max() <= 1e-11 * np.abs(du_o).max()
    assert np.abs(dc - dc_o).max() <= 1e-11 * np.abs(dc_o).max()

    def loss(uu, cc):
        with torch.no_grad():
            return 0.5 * float(((igatrim.mf_apply(plan, cc, uu) - ft) ** 2).sum())

    rng = np.random.default_rng(4)
    h = 0.1
    u0, c0 = ut.detach(), ct.detach()
    for _ in range(3):
        v = torch.as_tensor(rng.standard_normal(len(u)), device="cuda")
        fd = (loss(u0 + h * v, c0) - loss(u0 - h * v, c0)) / (2 * h)
        assert abs(fd - float(ut.grad @ v)) <= 1e-7 * abs(fd)
        w = torch.as_tensor(rng.standard_normal(len(c0)), device="cuda")
        fd = (loss(u0, c0 + h * w) - loss(u0, c0 - h * w)) / (2 * h)
        assert abs(fd - float(ct.grad @ w)) <= 1e-7 * abs(fd)
