"""Benchmark: trimmed-patch mass-matrix formation on one MI355X.

Step = one pass of the whole formation path on the device, from the raw
inputs (knot vectors, trimming curve, geometry control points) already in
HBM to the FP64 band matrix in HBM: weighted-quadrature layout and weights,
trimming (pieces, crossings, arcs, classes, compaction), cut-element rules,
c = |det J| at every rule point, interior rows (WQ + sum factorisation) and
cut rows (hybrid Gauss). Workload: degree 4, 256 x 256 elements, perturbed
geometry, hole bounded by a 16-point closed cubic B-spline (seeded).

Prints one JSON line. `value` = structural nonzeros formed per second.
Beside the headline the line carries: the same workload with discontinuous
weighted quadrature; 256 patches formed by the batched persistent kernel
(HIP graph, autotuned) against the same patches formed one by one; the
matrix-free product and its adjoint on 1024 x 1024 elements against plain
formation at that size; the dominant kernel's roofline; the oracle's rate on
a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--cpu-rows", type=int, default=8000, help="oracle sample: interior rows")
    ap.add_argument("--no-extra", action="store_true", help="headline only (no DWQ / batched / adjoint lines)")
    ap.add_argument("--batch", type=int, default=256, help="patches of the batched workload")
    ap.add_argument("--mf-N", type=int, default=1024, help="elements per direction of the matrix-free workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 5 times (scale of the HBM byte counters) and exit")
    return ap.parse_args()


def _timed(fn, steps, warmup, sync):
    """Mean milliseconds of fn() over `steps` calls after `warmup`, synchronised on both sides."""
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return 1e3 * (time.perf_counter() - t0) / steps


def _source_digest(sections):
    """Hash of the kernel's source: for each (file, title), the lines from the `// ---- title`
    section rule to the next rule (the whole file if title is None)."""
    import hashlib
    h = hashlib.sha256()
    for p, title in sections:
        with open(os.path.join(ROOT, p)) as fh:
            lines = fh.read().splitlines(True)
        if title is not None:
            start = [i for i, ln in enumerate(lines) if ln.startswith("// ---") and ln.rstrip().endswith(title)]
            if len(start) != 1:
                return None
            end = next((j for j in range(start[0] + 1, len(lines)) if lines[j].startswith("// ---")), len(lines))
            lines = lines[start[0]:end]
        h.update("".join(lines).encode())
    return h.hexdigest()[:16]


def _traffic(kernel_file, sources):
    """HBM bytes per launch from a committed counter summary, or None if the kernel changed since."""
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source digest") != _source_digest(sources):
        return None
    try:
        return int(float(vals["HBM bytes per launch"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, nnz_total, n_act, sample_rows):
    """The oracle (plain NumPy, as it stands) on a bounded sample of the same workload.

    Sample: its trimming + weight set-up on the full patch, then `sample_rows`
    interior rows (weighted-quadrature double sums) and a proportional share of
    the cut rows (element Gauss + cut rule). The rate is the sample's structural
    nonzeros over its time; set-up time is charged in proportion to the share of
    rows sampled.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.assemble import Oracle

    with threadpool_limits(limits=1):
        return _cpu_baseline(Oracle, np, cfg, nnz_total, n_act, sample_rows)


def _cpu_baseline(Oracle, np, cfg, nnz_total, n_act, sample_rows):
    t0 = time.perf_counter()
    o = Oracle(cfg)
    t_setup = time.perf_counter() - t0
    interior = o.interior_rows_flat()
    cut = o.cut_rows_flat()
    k_int = min(sample_rows, len(interior))
    frac = k_int / max(1, len(interior))
    k_cut = max(1, int(round(frac * len(cut))))
    rng = np.random.default_rng(0)
    ri = np.sort(rng.choice(interior, k_int, replace=False))
    rc = np.sort(rng.choice(cut, k_cut, replace=False))
    t1 = time.perf_counter()
    Mi = o.wq_rows(ri)
    # elements needed by the sampled cut rows
    p, ts = o.p, o.ts
    els = set()
    for f in rc:
        i2, i1 = divmod(int(f), ts.n1)
        for e2 in range(max(0, i2 - p), min(ts.N2 - 1, i2) + 1):
            for e1 in range(max(0, i1 - p), min(ts.N1 - 1, i1) + 1):
                if ts.ecls[e2, e1] != 0:
                    els.add((e2, e1))
    els = [(e1, e2) for (e2, e1) in sorted(els)]
    Mc = o.gauss_reference(rc, els)
    t_rows = time.perf_counter() - t1
    nnz_sample = Mi.nnz + Mc.nnz
    t_charged = t_rows + frac * t_setup
    return {"value": nnz_sample / t_charged, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"set-up on the full patch ({t_setup:.1f} s, charged x{frac:.3f}) + {k_int} interior rows "
                      f"+ {k_cut} cut rows of the same workload ({nnz_sample} nnz in {t_rows:.1f} s)"}


INTERIOR_SOURCES = [("paper_2101_08053_amd/csrc/form_body.hpp", "interior rows"),
                    ("paper_2101_08053_amd/csrc/form.hip", "interior rows"),
                    ("paper_2101_08053_amd/csrc/common.hpp", None)]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the formation path runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2101_08053_amd import igatrim
    from paper_2101_08053_amd import workloads as wl

    if not os.path.exists(igatrim.LIB_PATH):
        from paper_2101_08053_amd import build
        build.build()
    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        sync()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "copies": 5}), flush=True)
        return
    stream = torch.cuda.current_stream()
    cfg = wl.config2(N=args.N, p=args.p)
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    sz = plan.sizes
    coef = plan.coeff()
    vals = torch.empty((sz["band"], sz["n_act"]), dtype=torch.float64, device="cuda")

    def step(full=True):
        plan.mass_form(coef, out=vals, full=full, stream=stream)

    for _ in range(args.warmup):
        step()
    sync()
    plan.status()

    # timed region: the whole formation path (the library replays it as one HIP graph from the
    # second identical call on; the warm-up steps record it)
    ms_step = _timed(step, args.steps, 0, sync)
    nnz = sz["nnz"]
    value = nnz / (ms_step * 1e-3)
    ms_form = _timed(lambda: step(full=False), args.steps, 2, sync)
    # the same step launched kernel by kernel on the two streams, then with per-phase HIP events
    # on the streams the kernels run on (the interior kernel then runs alone and its events
    # bracket its dispatch)
    plan.set_graph(False)
    ms_eager = _timed(step, args.steps, 2, sync)
    plan.set_timing(True)
    ms_timed = _timed(step, args.steps, 0, sync)
    phases = plan.timings()
    plan.set_timing(False)
    plan.set_graph(True)

    # dominant kernel of the formation: interior rows (one k_interior launch per step), HBM bound
    int_ms, int_cnt = phases["interior"]
    k_ms = int_ms / max(1, int_cnt)
    alg_bytes = 8 * sz["band"] * sz["n_interior"] + 8 * sz["q1"] * sz["q2"]
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = _traffic(f"k_interior_p{args.p}_N{args.N}_traffic.md", INTERIOR_SOURCES)
    roof = {"kernel": f"k_interior<{args.p}> (interior rows: WQ + sum factorisation)", "bound": "hbm",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_ms": round(k_ms, 5), "algorithmic_bytes": int(alg_bytes),
            "timing": "HIP events at the kernel's dispatch start and end, every step of the pass with phase "
                      "events (the kernel runs alone there)"}

    out = {
        "metric": "mass-matrix nnz formed/s (FP64, p=4 trimmed 256^2)",
        "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"trimmed patch p={args.p}, {args.N}x{args.N} elements, perturbed geometry "
                               "c=|det J|, 16-point cubic B-spline hole, hybrid Gauss, whole formation path",
                   "p": args.p, "elements": [args.N, args.N], "n_act": sz["n_act"], "nnz": nnz,
                   "n_interior": sz["n_interior"], "n_cut_fn": sz["n_cut_fn"], "n_cut_el": sz["n_cut_el"],
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": None,
        "launches": {"graph_ms_per_step": ms_step, "kernel_by_kernel_ms_per_step": ms_eager,
                     "with_phase_events_ms_per_step": ms_timed},
        # a phase's event pairs summed over the timed pass (a phase may run on both streams: the
        # pairs overlap, so the phases need not add up to the step)
        "phases_ms_per_step": {k: round(v[0] / args.steps, 5) for k, v in phases.items()},
        "formation_only": {"ms_per_step": ms_form, "value": nnz / (ms_form * 1e-3), "unit": "nnz/s",
                           "note": "tables resident; coefficient + interior rows + cut rows"},
    }
    del vals
    if not args.no_extra:
        out["dwq"] = bench_dwq(igatrim, wl, cfg, args, sync, stream)
        out["projection"] = bench_projection(igatrim, wl, cfg, args, sync)
        out["batched"] = bench_batched(igatrim, wl, args, sync)
        out["adjoint"] = bench_adjoint(igatrim, wl, args, sync)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, nnz, sz["n_act"], args.cpu_rows)
    print(json.dumps(out), flush=True)


def bench_dwq(igatrim, wl, cfg, args, sync, stream):
    """The headline workload with discontinuous weighted quadrature for the cut rows."""
    import torch
    plan = igatrim.Plan(cfg, igatrim.DWQ)
    sz = plan.sizes
    coef = plan.coeff()
    vals = torch.empty((sz["band"], sz["n_act"]), dtype=torch.float64, device="cuda")
    ms_full = _timed(lambda: plan.mass_form(coef, out=vals, full=True, stream=stream), args.steps, args.warmup, sync)
    ms_form = _timed(lambda: plan.mass_form(coef, out=vals, stream=stream), args.steps, 2, sync)
    plan.status()
    return {"value": sz["nnz"] / (ms_full * 1e-3), "unit": "nnz/s", "ms_per_step": ms_full,
            "formation_only_ms": ms_form, "formation_only_value": sz["nnz"] / (ms_form * 1e-3),
            "n_dwq_rows": sz["n_dwq_rows"], "n_cut_fn": sz["n_cut_fn"],
            "note": "same workload and step as the headline, cut rows by DWQ boxes + element rules"}


def bench_projection(igatrim, wl, cfg, args, sync):
    """L2 projection (right-hand side + Jacobi PCG to 1e-12) on the headline workload's matrix."""
    import math
    import torch
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    sz = plan.sizes
    coef = plan.coeff()
    vals = plan.mass_form(coef, full=True)
    g = igatrim.target_sincos(2.0, 0.0, 3.0, 0.0)  # sin(2x) cos(3y), the paper's target
    igatrim.l2_project(plan, vals, coef, g, rtol=1e-12)  # warm-up: workspace allocation
    sync()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        u, info = igatrim.l2_project(plan, vals, coef, g, rtol=1e-12)
    sync()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    it = max(1, info["iterations"])
    # per iteration: the band values (symmetrised matrix) once, and about seven vectors
    bytes_it = 8 * sz["band"] * sz["n_act"] + 7 * 8 * sz["n_act"]
    return {"ms": ms, "iterations": info["iterations"], "rel_residual": info["rel_residual"],
            "ms_per_iteration": ms / it, "spmv_GBs_per_iteration": bytes_it / (ms / it * 1e-3) / 1e9,
            "frac_of_hbm_peak": bytes_it / (ms / it * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "note": "target g = sin(2x) cos(3y), c = |det J|; rhs + symmetrisation + Jacobi PCG, synchronous; "
                    "bytes per iteration = band values + 7 vectors"}


def bench_batched(igatrim, wl, args, sync):
    """256 patches (p 2..5, 16..256 elements per direction, one ellipse each): batched vs one by one."""
    import torch
    cfgs = wl.config4(n_patch=args.batch)
    t0 = time.perf_counter()
    plans = [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]
    t_plan = time.perf_counter() - t0
    coeffs = [p.coeff() for p in plans]
    nnz = sum(p.sizes["nnz"] for p in plans)
    b = igatrim.Batch(plans, coeffs)
    tune_ms = b.autotune()
    steps = max(5, args.steps // 2)
    ms_graph = _timed(lambda: b.form(use_graph=True), steps, 2, sync)
    ms_eager = _timed(lambda: b.form(use_graph=False), steps, 2, sync)
    b.status()
    outs = b.outs

    def plain():
        for p, c, o in zip(plans, coeffs, outs):
            p.mass_form(c, out=o)

    ms_plain = _timed(plain, max(3, steps // 2), 2, sync)  # the second call records each plan's graph
    info = b.info()
    return {"value": nnz / (ms_graph * 1e-3), "unit": "nnz/s", "ms": ms_graph, "eager_ms": ms_eager,
            "plain_ms": ms_plain, "plain_value": nnz / (ms_plain * 1e-3), "speedup_vs_plain": ms_plain / ms_graph,
            "patches": len(plans), "nnz": nnz, "items": info["n_items"], "grid": info["grid"],
            "wg_per_cu": info["wg_per_cu"], "chunk": info["chunk"],
            "registers": "256 (two workgroups per CU)" if info["capped"] else "up to 512 (one workgroup per CU)",
            "order": ["cost-sorted", "patch by patch"][info["order"]],
            "cut_elements": "persistent queue" if info["grid"] > 0 else "one workgroup each (autotuner's choice)",
            "autotune_best_ms": tune_ms, "plan_setup_s": round(t_plan, 2),
            "note": "formation over resident tables, one graph replay per call (cut element matrices beside "
                    "per-degree coefficient and interior launches, then the element-formed rows) vs one formation "
                    "call per patch"}


def bench_adjoint(igatrim, wl, args, sync):
    """Matrix-free y = M(c) u and its adjoint on the 1024^2 workload, against plain formation there."""
    import torch
    cfg = wl.config5(N=args.mf_N)
    plan = igatrim.Plan(cfg, igatrim.HYBRID_GAUSS)
    sz = plan.sizes
    pts = plan.points()
    c = wl.config5_coef(pts[:, 0], pts[:, 1], torch).contiguous()
    u_np, f_np = wl.config5_vectors(sz["n_act"])
    u = torch.as_tensor(u_np, device="cuda")
    gy = torch.as_tensor(f_np, device="cuda")
    steps = max(5, args.steps // 2)
    ms_fwd = _timed(lambda: igatrim.mf_apply(plan, c, u), steps, 2, sync)
    ms_bwd = _timed(lambda: igatrim.mf_adjoint(plan, c, u, gy), steps, 2, sync)
    coef = plan.coeff(igatrim.COEF_AT_POINTS, c_points=c)
    vals = torch.empty((sz["band"], sz["n_act"]), dtype=torch.float64, device="cuda")
    ms_form = _timed(lambda: plan.mass_form(coef, out=vals), steps, 2, sync)
    nnz = sz["nnz"]
    return {"forward_ms": ms_fwd, "backward_ms": ms_bwd, "plain_formation_ms": ms_form,
            "forward_value": nnz / (ms_fwd * 1e-3), "backward_value": nnz / (ms_bwd * 1e-3),
            "plain_value": nnz / (ms_form * 1e-3), "unit": "nnz-equivalent/s", "nnz": nnz,
            "n_act": sz["n_act"], "n_points": sz["n_points"],
            "note": f"p=4, {args.mf_N}^2 elements, c at every rule point; y = M(c)u and (dL/du, dL/dc)"}


if __name__ == "__main__":
    main()
