"""Batched L2 projection (Sect. 4.2) of a batch's patches: right-hand sides and Jacobi-PCG for
every patch in the same launches.

Each patch's step sizes come from its own block partials, summed in the
one-patch solver's order, and its convergence is tested at the one-patch
solver's iterations, so every patch's solution and iteration count must equal
iga_trim_l2_project's on the same matrix bit for bit. The one-patch
projection is checked against the oracle in test_gpu_solve; here the oracle's
residual of the batched solutions is checked as well, on small patches of the
batched workload's generator (degrees 2..5, element counts log-uniform per
direction, one ellipse each, c = |det J|, g = sin(pi x) cos(pi y) at physical
points).
"""
import math

import numpy as np
import pytest

from gpu_common import require_gpu, say
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sincos(igatrim):
    return igatrim.target_sincos(math.pi, 0.0, math.pi, 0.0)


def _batch(n, n_range, seed, p_range=None):
    from paper_2101_08053_amd import igatrim
    kw = {"seed": seed}
    if p_range is not None:
        kw["p_range"] = p_range
    cfgs = wl.config4(n_patch=n, n_range=n_range, **kw)
    plans = [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]
    coeffs = [p.coeff() for p in plans]
    b = igatrim.Batch(plans, coeffs)
    b.form(use_graph=True)
    b.status()
    return cfgs, plans, coeffs, b


def test_batch_project_equals_one_patch():
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs, plans, coeffs, b = _batch(10, (6, 40), wl.SEED_BASE + 50)
    say("[batch project] degrees", [c.p for c in cfgs], "sizes", [c.n_el for c in cfgs])
    g = _sincos(igatrim)
    us, infos = b.project([g] * len(plans), rtol=1e-12)
    for k, (p, c, o) in enumerate(zip(plans, coeffs, b.outs)):
        u1, info1 = igatrim.l2_project(p, o, c, g, rtol=1e-12)
        say(f"   patch {k}: p={p.sizes['p']} n_act={p.sizes['n_act']} batched {infos[k]} one-patch {info1}")
        assert infos[k]["converged"] and infos[k]["rel_residual"] <= 1e-12
        assert infos[k]["iterations"] == info1["iterations"]
        assert infos[k]["rel_residual"] == info1["rel_residual"]
        assert np.array_equal(us[k].cpu().numpy(), u1.cpu().numpy()), f"patch {k}"


def test_batch_project_against_oracle():
    """The oracle's residual ||b - A u|| / ||b|| of each batched solution, with the oracle's own
    (hybrid Gauss) matrix and right-hand side, stays within 1e-9 (PCG stops at 1e-12 on the
    device's A and b; the two differ by the end-to-end rule differences)."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    from oracle import project
    from oracle.assemble import Oracle
    cfgs, plans, coeffs, b = _batch(4, (8, 18), wl.SEED_BASE + 51)
    us, infos = b.project([_sincos(igatrim)] * len(plans), rtol=1e-12)
    for k, cfg in enumerate(cfgs):
        o = Oracle(cfg)
        M = o.hybrid()
        bo = project.rhs(o, wl.config1_target)
        u = us[k].cpu().numpy()
        res = np.linalg.norm(bo - 0.5 * (M + M.T) @ u) / np.linalg.norm(bo)
        say(f"[batch project oracle] patch {k} p={cfg.p} N={cfg.n_el}: {infos[k]} oracle residual {res:.2e}")
        assert infos[k]["converged"]
        assert res <= 1e-9


def test_batch_project_mixed_convergence():
    """A zero target (b = 0: converged before the first iteration, u stays the start vector)
    beside ordinary ones, and a start vector that is already the solution."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs, plans, coeffs, b = _batch(5, (6, 30), wl.SEED_BASE + 52)
    zero = igatrim.target_sincos(0.0, 0.0, 0.0, 0.0)
    targets = [zero if k % 2 else _sincos(igatrim) for k in range(len(plans))]
    us, infos = b.project(targets, rtol=1e-12)
    for k in range(len(plans)):
        if k % 2:
            assert infos[k]["iterations"] == 0 and infos[k]["converged"]
            assert not np.any(us[k].cpu().numpy())
        else:
            assert infos[k]["converged"] and infos[k]["iterations"] > 0
    us2, infos2 = b.project(targets, rtol=1e-10, u0=us)
    say("[batch project restart] iterations", [i["iterations"] for i in infos2])
    assert all(i["converged"] and i["iterations"] == 0 for i in infos2)


def test_batch_project_noconv_status():
    """maxit smaller than the iterations needed: IGA_E_NOCONV, every patch reports maxit."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs, plans, coeffs, b = _batch(3, (10, 24), wl.SEED_BASE + 53)
    with pytest.raises(igatrim.IgaError) as ei:
        b.project([_sincos(igatrim)] * len(plans), rtol=1e-12, maxit=3)
    assert ei.value.code == -8
    us, infos = b.project([_sincos(igatrim)] * len(plans), rtol=1e-12, maxit=3, raise_on_noconv=False)
    assert all(i["iterations"] == 3 and not i["converged"] for i in infos)
    for k, (p, c, o) in enumerate(zip(plans, coeffs, b.outs)):
        u1, info1 = igatrim.l2_project(p, o, c, _sincos(igatrim), rtol=1e-12, maxit=3, raise_on_noconv=False)
        assert info1["iterations"] == 3
        assert np.array_equal(us[k].cpu().numpy(), u1.cpu().numpy())


def test_batch_project_degree_ends():
    """Degrees 1 and 6 in one batch: bit for bit the one-patch projections."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs = (wl.config4(n_patch=2, n_range=(8, 24), p_range=(1, 1), seed=wl.SEED_BASE + 54)
            + wl.config4(n_patch=2, n_range=(12, 24), p_range=(6, 6), seed=wl.SEED_BASE + 55))
    plans = [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]
    plans.append(igatrim.Plan(cfgs[0], igatrim.GAUSS_REF))
    coeffs = [p.coeff() for p in plans]
    b = igatrim.Batch(plans, coeffs)
    b.form()
    g = _sincos(igatrim)
    us, infos = b.project([g] * len(plans), rtol=1e-12)
    for k, (p, c, o) in enumerate(zip(plans, coeffs, b.outs)):
        u1, info1 = igatrim.l2_project(p, o, c, g, rtol=1e-12)
        assert infos[k]["iterations"] == info1["iterations"]
        assert np.array_equal(us[k].cpu().numpy(), u1.cpu().numpy()), f"patch {k}"


def test_batch_project_with_dwq_plans():
    """DWQ plans beside hybrid Gauss ones: box parts of the right-hand side in the same launches,
    bit for bit the one-patch projections."""
    require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs = wl.config4(n_patch=6, n_range=(8, 32), seed=wl.SEED_BASE + 56)
    plans = [igatrim.Plan(c, igatrim.DWQ if k % 2 == 0 else igatrim.HYBRID_GAUSS) for k, c in enumerate(cfgs)]
    coeffs = [p.coeff() for p in plans]
    b = igatrim.Batch(plans, coeffs)
    b.form(use_graph=True)
    b.status()
    g = _sincos(igatrim)
    us, infos = b.project([g] * len(plans), rtol=1e-12)
    for k, (p, c, o) in enumerate(zip(plans, coeffs, b.outs)):
        u1, info1 = igatrim.l2_project(p, o, c, g, rtol=1e-12)
        say(f"   patch {k}: method={p.method} p={p.sizes['p']} n_dwq_rows={p.sizes['n_dwq_rows']} "
            f"batched {infos[k]} one-patch {info1}")
        assert infos[k]["converged"]
        assert infos[k]["iterations"] == info1["iterations"]
        assert np.array_equal(us[k].cpu().numpy(), u1.cpu().numpy()), f"patch {k}"
