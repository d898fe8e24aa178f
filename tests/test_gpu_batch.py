"""Batched formation (a persistent launch of the cut element matrices, per-degree launches of the
coefficients, interior tiles and element-formed rows on two streams, HIP graph, autotuner).

The batched launches run the same bodies as the one-patch kernels, with the
same summation order per entry, so their output must equal the one-patch
formation bit for bit; the one-patch formation itself is checked
against the oracle in test_gpu_form. The patch set follows the batched
workload's generator (degrees 2..5, element counts log-uniform per
direction, one ellipse each) at sizes small enough for a test.
"""
import numpy as np
import pytest

from gpu_common import require_gpu, say
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _plans(n=10, n_range=(6, 40), seed=None):
    from paper_2101_08053_amd import igatrim
    kw = {} if seed is None else {"seed": seed}
    cfgs = wl.config4(n_patch=n, n_range=n_range, **kw)
    return cfgs, [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]


def _plain(plans, coeffs):
    return [p.mass_form(c).cpu().numpy() for p, c in zip(plans, coeffs)]


def test_batch_equals_plain():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs, plans = _plans()
    say("[batch] degrees", [c.p for c in cfgs], "sizes", [c.n_el for c in cfgs])
    coeffs = [p.coeff() for p in plans]
    ref = _plain(plans, coeffs)
    b = igatrim.Batch(plans, coeffs)
    for o in b.outs:
        o.fill_(np.nan)
    outs = [o.cpu().numpy() for o in b.form()]
    b.status()
    for k, (g, r) in enumerate(zip(outs, ref)):
        assert np.array_equal(g, r), f"patch {k}: max diff {np.nanmax(np.abs(g - r))}"
    info = b.info()
    say("[batch] info", info)
    assert info["n_plans"] == len(plans) and info["grid"] >= 1


def test_batch_graph_replays():
    """Graph replays, with eager work and synchronisation between them, equal the eager batch."""
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs, plans = _plans(n=8, seed=wl.SEED_BASE + 40)
    coeffs = [p.coeff() for p in plans]
    ref = _plain(plans, coeffs)
    b = igatrim.Batch(plans, coeffs)
    for rep in range(4):
        for o in b.outs:
            o.zero_()
        x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
        _ = (x * x).sum().item()           # eager work between replays
        torch.cuda.synchronize()
        b.form(use_graph=True)
        torch.cuda.synchronize()
        b.status()
        for k, (o, r) in enumerate(zip(b.outs, ref)):
            assert np.array_equal(o.cpu().numpy(), r), f"replay {rep} patch {k}"
    assert b.info()["graph_ready"] == 1


def test_batch_autotune_keeps_results():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs, plans = _plans(n=12, seed=wl.SEED_BASE + 41)
    coeffs = [p.coeff() for p in plans]
    ref = _plain(plans, coeffs)
    b = igatrim.Batch(plans, coeffs)
    ms = b.autotune()
    info = b.info()
    say(f"[batch autotune] best {ms:.3f} ms, {info}")
    assert info["wg_per_cu"] in (1, 2, 4, 8, 12, 16) and info["order"] in (0, 1)
    outs = [o.cpu().numpy() for o in b.form(use_graph=True)]
    b.status()
    for g, r in zip(outs, ref):
        assert np.array_equal(g, r)


def test_batch_constant_coefficient_and_one_shot():
    """c = 1 (no coefficient items) through the one-shot call; area invariant per patch."""
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    from oracle.trim import TrimmedSpace
    cfgs, plans = _plans(n=6, seed=wl.SEED_BASE + 42)
    coeffs = [p.coeff(igatrim.COEF_CONST, 1.0) for p in plans]
    ref = _plain(plans, coeffs)
    outs = [o.cpu().numpy() for o in igatrim.mass_form_batched(plans, coeffs)]
    for g, r, c in zip(outs, ref, cfgs):
        assert np.array_equal(g, r)
        assert abs(g.sum() - TrimmedSpace(c).visible_area()) < 1e-10


def test_batch_degree_ends_and_element_gauss():
    """Degrees 1 and 6 (the ends of what the batch takes, outside the workload's 2..5) and an
    element-Gauss plan (every row formed element-wise, no interior tiles) in one batch, eager and
    replayed: bit for bit the one-patch formations."""
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs = (wl.config4(n_patch=3, n_range=(8, 30), p_range=(1, 1), seed=wl.SEED_BASE + 43)
            + wl.config4(n_patch=3, n_range=(12, 30), p_range=(6, 6), seed=wl.SEED_BASE + 44))
    say("[batch ends] degrees", [c.p for c in cfgs], "sizes", [c.n_el for c in cfgs])
    plans = [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]
    plans.append(igatrim.Plan(cfgs[0], igatrim.GAUSS_REF))
    coeffs = [p.coeff() for p in plans]
    ref = _plain(plans, coeffs)
    b = igatrim.Batch(plans, coeffs)
    for use_graph in (False, True, True):
        for o in b.outs:
            o.fill_(np.nan)
        outs = [o.cpu().numpy() for o in b.form(use_graph=use_graph)]
        b.status()
        for k, (g, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(g, r), f"patch {k} (p = {plans[k].sizes['p']}), graph {use_graph}"


def test_batch_with_dwq_plans():
    """DWQ plans in a batch (Sect. 3.3): the side rules of every DWQ patch solved in one launch per
    degree, the box parts added after the element-formed rows; eager and replayed, each patch equals
    its one-patch formation bit for bit (degree 5 patches as DWQ as in the batched workload, plus
    degrees 2 and 6 and a constant coefficient)."""
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfgs = wl.config4(n_patch=10, n_range=(8, 40), seed=wl.SEED_BASE + 45)
    cfgs += wl.config4(n_patch=2, n_range=(10, 24), p_range=(6, 6), seed=wl.SEED_BASE + 46)
    cfgs += wl.config4(n_patch=2, n_range=(10, 24), p_range=(2, 2), seed=wl.SEED_BASE + 47)
    methods = [igatrim.DWQ if (c.p in (5, 6) or k >= len(cfgs) - 2) else igatrim.HYBRID_GAUSS
               for k, c in enumerate(cfgs)]
    plans = [igatrim.Plan(c, m) for c, m in zip(cfgs, methods)]
    coeffs = [p.coeff() for p in plans]
    coeffs[-1] = plans[-1].coeff(igatrim.COEF_CONST, 1.0)
    say("[batch dwq] degrees", [c.p for c in cfgs], "methods", methods,
        "dwq rows", [p.sizes["n_dwq_rows"] for p in plans])
    assert any(p.sizes["n_dwq_rows"] > 0 for p in plans)
    ref = _plain(plans, coeffs)
    b = igatrim.Batch(plans, coeffs)
    for use_graph in (False, True, True):
        for o in b.outs:
            o.fill_(np.nan)
        outs = [o.cpu().numpy() for o in b.form(use_graph=use_graph)]
        b.status()
        for k, (g, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(g, r), f"patch {k} (p = {cfgs[k].p}, method {methods[k]}), graph {use_graph}"
    ms = b.autotune()
    outs = [o.cpu().numpy() for o in b.form(use_graph=True)]
    b.status()
    for g, r in zip(outs, ref):
        assert np.array_equal(g, r)
