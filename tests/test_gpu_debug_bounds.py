"""The index-checking build (band stores' slot and row checked, -DIGA_DEBUG_BOUNDS) counts no out-of-range store.

A child process loads libigatrim_debug.so (IGA_TRIM_LIB) and runs the
formation paths that store into the band layout and the per-row scratch
arrays: hybrid and element-Gauss full formations with c = |det J| (interior
rows, inside sums and cut entries of the element-formed rows), naive WQ (end
rows of every active function), DWQ at p = 4 (box parts in scratch) and p = 6
(box parts added to the band), a batch of mixed degrees with DWQ patches, and
the projection. Every store checks its slot and row; the count must stay 0.
The checking build is made on the host beside the release one
(`__graft_entry__.build()`).
"""
import os
import subprocess
import sys

import pytest

from gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_2101_08053_amd", "libigatrim_debug.so")

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_2101_08053_amd import igatrim
from paper_2101_08053_amd import workloads as wl
assert igatrim.LIB_PATH.endswith("libigatrim_debug.so"), igatrim.LIB_PATH
torch.cuda.set_device(0)
igatrim.debug_bounds_hits(reset=True)
cases = [("hybrid config2 N48 p4", wl.config2(N=48, p=4), igatrim.HYBRID_GAUSS),
         ("element Gauss config2 N32 p3", wl.config2(N=32, p=3), igatrim.GAUSS_REF),
         ("naive WQ config1 N24", wl.config1(N=24), igatrim.NAIVE_WQ),
         ("DWQ config2 N48 p4", wl.config2(N=48, p=4), igatrim.DWQ),
         ("DWQ config3 N40 p6", wl.config3(N=40), igatrim.DWQ)]
for name, cfg, method in cases:
    plan = igatrim.Plan(cfg, method)
    c = plan.coeff()
    for full in (True, False, True):
        plan.mass_form(c, full=full)
    plan.set_graph(False)
    vals = plan.mass_form(c, full=True)
    plan.status()
    if method != igatrim.NAIVE_WQ:
        igatrim.l2_project(plan, vals, c, igatrim.target_sincos(2.0, 0.0, 3.0, 0.0), rtol=1e-10)
    print(name, "hits", igatrim.debug_bounds_hits(), flush=True)
cfgs = wl.config4(n_patch=6, n_range=(16, 40))
plans = [igatrim.Plan(cfg, igatrim.DWQ if cfg.p == 5 else igatrim.HYBRID_GAUSS) for cfg in cfgs]
b = igatrim.Batch(plans, [p.coeff() for p in plans])
for use_graph in (False, True, True):
    b.form(use_graph=use_graph)
b.status()
print("batch of", len(plans), "hits", igatrim.debug_bounds_hits(), flush=True)
print("total", igatrim.debug_bounds_hits(), flush=True)
"""


def test_debug_build_counts_no_out_of_range_store():
    require_gpu()
    if not os.path.exists(DEBUG_LIB):
        pytest.skip("libigatrim_debug.so is not built (__graft_entry__.build() makes it)")
    env = dict(os.environ, IGA_TRIM_LIB=DEBUG_LIB)
    say("[debug bounds] child process on", DEBUG_LIB)
    r = subprocess.run([sys.executable, "-u", "-c", CHILD, ROOT], capture_output=True, text=True, env=env,
                       timeout=240)
    say(r.stdout[-3000:])
    assert r.returncode == 0, r.stderr[-4000:]
    lines = [ln for ln in r.stdout.splitlines() if " hits " in ln or ln.startswith("total")]
    assert len(lines) == 7, r.stdout
    for ln in lines:
        assert ln.split()[-1] == "0", ln
