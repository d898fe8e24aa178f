"""Allocation-free matrix-free product (iga_mf_apply_noalloc) against iga_mf_apply.

Both run the same kernels; the allocation-free call takes its intermediate
arrays from the library's static scratch array instead of the plan's
workspace, so the products must agree bit for bit. Two calls in a row, the
second on a smaller patch (the scratch keeps the first call's contents), and
a patch too large for the scratch array (a clear IGA_E_CAPACITY error).
"""
import numpy as np
import pytest

from gpu_common import require_gpu, say
from paper_2101_08053_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _noalloc(plan, c, u, y):
    """The C entry point through the binding; returns its status code."""
    from paper_2101_08053_amd import igatrim
    try:
        igatrim.mf_apply_noalloc(plan, c, u, y)
    except igatrim.IgaError as e:
        return e.code
    return 0


def _case(N, seed_shift):
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    cfg = wl.config5(N=N)
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    pts = plan.points()
    c = wl.config5_coef(pts[:, 0], pts[:, 1], torch).contiguous()
    rng = np.random.default_rng(wl.SEED_BASE + 60 + seed_shift)
    u = torch.as_tensor(rng.standard_normal(plan.sizes["n_act"]), device="cuda")
    return plan, c, u


def test_noalloc_equals_apply_twice():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    for N, shift in ((96, 0), (40, 1)):  # the second patch is smaller
        plan, c, u = _case(N, shift)
        y_ref = igatrim.mf_apply(plan, c, u)
        y = torch.full_like(y_ref, float("nan"))
        code = _noalloc(plan, c, u, y)
        assert code == 0, igatrim.lib().iga_last_error().decode()
        torch.cuda.synchronize()
        say(f"[noalloc] N={N} n_act={plan.sizes['n_act']} max |y - y_ref| = "
            f"{float((y - y_ref).abs().max()):.3e}")
        assert torch.equal(y, y_ref)
        plan.close()


def test_noalloc_rejects_oversized_patch():
    torch = require_gpu()
    from paper_2101_08053_amd import igatrim
    plan, c, u = _case(2000, 2)  # needs about 16 MB of band rows and 10 MB of element vectors
    y = torch.zeros_like(u)
    code = _noalloc(plan, c, u, y)
    msg = igatrim.lib().iga_last_error().decode()
    say(f"[noalloc] N=2000: code {code}: {msg}")
    assert code == -7 and "scratch" in msg
    assert not torch.any(y)
