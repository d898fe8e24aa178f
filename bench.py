"""Benchmark: trimmed-patch mass-matrix formation on one MI355X.

Step = one pass of the whole formation path on the device, from the raw
inputs (knot vectors, trimming curve, geometry control points) already in
HBM to the FP64 band matrix in HBM: weighted-quadrature layout and weights,
trimming (pieces, crossings, arcs, classes, compaction), cut-element rules,
c = |det J| at every rule point, interior rows (WQ + sum factorisation) and
cut rows (hybrid Gauss). Workload: degree 4, 256 x 256 elements, perturbed
geometry, hole bounded by a 16-point closed cubic B-spline (seeded).

Prints one JSON line. `value` = structural nonzeros formed per second.
`roofline` is the kernel with the largest time per step, from a pass in
which every dispatch is bracketed by HIP events on its own stream; beside it
`kernels` lists every kernel of the step and `rooflines` the per-section
objects. The line also carries: the measured copy / FP64 FMA / FP64 MFMA
ceilings; the step with a 1 GiB write between replays (the step's 32 MB
would otherwise stay in the 256 MB last-level cache); the same workload with
discontinuous weighted quadrature (with its own rooflines); the degree-6,
512 x 512, three-ellipse DWQ workload; the L2 projection, in the trimmed
basis and in the extended B-spline basis; 256 patches formed by the batched
launches (HIP graph, autotuned) and L2-projected by the batched PCG, against
the same patches one by one; the matrix-free product and its adjoint on
1024 x 1024 elements against plain formation there; Table 1 (the methods
against element Gauss, p = 1..8) from the device; and the oracle's rate on a
bounded sample, on one core and on all host cores.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6      # vector and matrix core (dense) alike


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--cpu-rows", type=int, default=8000, help="oracle sample: interior rows per process")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes for the all-core sample (0: host cores, "
                                                              "at most 16)")
    ap.add_argument("--no-extra", action="store_true", help="headline only (no other sections)")
    ap.add_argument("--sections", default="dwq,config3_dwq,projection,batched,adjoint,table1",
                    help="comma-separated sections after the headline")
    ap.add_argument("--batch", type=int, default=256, help="patches of the batched workload")
    ap.add_argument("--mf-N", type=int, default=1024, help="elements per direction of the matrix-free workload")
    ap.add_argument("--cfg3-N", type=int, default=512, help="elements per direction of the degree-6 DWQ workload")
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


# committed counter summaries per (p, N) workload
TRAFFIC_FILES = {(4, 256): "formation_p4_N256_hbm_traffic.md", (4, 1024): "matfree_p4_N1024_hbm_traffic.md"}
# the source sections each counted kernel is built from (counter values are used while they hash the same)
KERNEL_SOURCES = {
    "k_interior": [("paper_2101_08053_amd/csrc/form_body.hpp", "interior rows"),
                   ("paper_2101_08053_amd/csrc/form.hip", "interior rows"),
                   ("paper_2101_08053_amd/csrc/form_body.hpp", "coefficient"),
                   ("paper_2101_08053_amd/csrc/common.hpp", None)],
    "k_weights_coef": [("paper_2101_08053_amd/csrc/setup.hip", "WQ weights (5)"),
                       ("paper_2101_08053_amd/csrc/form_body.hpp", "coefficient"),
                       ("paper_2101_08053_amd/csrc/plan.hpp", None),
                       ("paper_2101_08053_amd/csrc/common.hpp", None)],
    "k_cut_rows": [("paper_2101_08053_amd/csrc/form_body.hpp", "cut rows"),
                   ("paper_2101_08053_amd/csrc/form.hip", "cut element matrices / rows"),
                   ("paper_2101_08053_amd/csrc/common.hpp", None)],
    "k_cut_elem": [("paper_2101_08053_amd/csrc/form_body.hpp", "cut element matrices"),
                   ("paper_2101_08053_amd/csrc/form.hip", "cut element matrices / rows"),
                   ("paper_2101_08053_amd/csrc/common.hpp", None)],
    "k_cutprep": [("paper_2101_08053_amd/csrc/trim.hip", "cut-element rules"),
                  ("paper_2101_08053_amd/csrc/trim.hip", "evaluation"),
                  ("paper_2101_08053_amd/csrc/plan.hpp", None),
                  ("paper_2101_08053_amd/csrc/common.hpp", None)],
    "k_mf_fwd": [("paper_2101_08053_amd/csrc/matfree.hip", None),
                 ("paper_2101_08053_amd/csrc/plan.hpp", None),
                 ("paper_2101_08053_amd/csrc/common.hpp", None)],
    "k_mf_adj": [("paper_2101_08053_amd/csrc/matfree.hip", None),
                 ("paper_2101_08053_amd/csrc/plan.hpp", None),
                 ("paper_2101_08053_amd/csrc/common.hpp", None)],
}


def _traffic(kernel, p=4, N=256):
    """HBM bytes per launch of `kernel` from the committed counter summary of its workload (p, N x N),
    or None if there is none for this kernel or the kernel's sources changed since."""
    base = kernel.split("<")[0]
    if (p, N) not in TRAFFIC_FILES or base not in KERNEL_SOURCES:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[(p, N)])
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get(f"{kernel} source digest") != _source_digest(KERNEL_SOURCES[base]):
        return None
    try:
        return int(float(vals[f"{kernel} HBM bytes per launch"]))
    except (KeyError, ValueError):
        return None


# ----------------------------------------------------------------- rooflines
def _roof(kernel, bound, work, ms, peaks, unit_work, note, traffic=None):
    """Roofline object: achieved = algorithmic work per launch / mean launch time."""
    if bound == "hbm":
        achieved = work / (ms * 1e-3) / 1e9
        peak, unit, meas = HBM_PEAK_GBS, "GB/s", peaks.get("copy_GBs")
    else:
        achieved = work / (ms * 1e-3) / 1e12
        peak, unit = FP64_PEAK_TFS, "TFLOP/s"
        meas = peaks.get("mfma_f64_TFs" if bound == "mfma" else "fma_f64_TFs")
    out = {"kernel": kernel, "bound": bound, "achieved": round(achieved, 4 if achieved < 10 else 1), "peak": peak,
           "unit": unit, "frac": round(achieved / peak, 5), "traffic": traffic, "avg_launch_ms": round(ms, 5),
           "algorithmic_" + ("bytes" if bound == "hbm" else "flops"): int(work),
           "per_unit": unit_work, "note": note}
    if meas:
        out["measured_peak"] = round(meas, 1)
        out["frac_of_measured"] = round(achieved / meas, 5)
    return out


def kernel_work(name, sz, plan_info):
    """(bound, algorithmic work per launch, per-unit statement) of a formation kernel, or None.

    Per-unit figures: interior rows write 8 (2p+1)^2 B each and read c on the
    WQ grid once (8 B per point); a cut element's Gram product sum_n w c phi phi^T
    costs n_nodes L (L+1)/2 FMA (upper triangle, L = (p+1)^2, 2 flops each);
    c = |det J| at a point writes 8 B (and, in a full formation, the point's
    coordinates, 16 B) and reads the control points (counted once per launch:
    16 n1 n2 B; a full formation computes the WQ grid's values beside the weight
    systems, k_weights_coef, and the band Gauss points' in the interior launch); a weight
    system of Eq. (5) (m = 2p+1 rows, q = 2p+2 points) is a Householder QR of
    q x m: 2 q m^2 - (2/3) m^3 flops; the cut-element preparation writes each
    node's (x, y, w) (24 B); the element-formed rows' cut entries read each cut
    element matrix once (8 L^2 B) and write their rows (8 (2p+1)^2 B); a DWQ
    row's box part is one value per slot (8 (2p+1)^2 B).
    """
    p = sz["p"]
    L = (p + 1) ** 2
    W2 = (2 * p + 1) ** 2
    base = name.split("<")[0]
    if base == "k_interior":
        work = 8 * W2 * sz["n_interior"] + 8 * sz["q1"] * sz["q2"]
        per = f"8 (2p+1)^2 = {8 * W2} B per interior row + 8 B per WQ point"
        if "coef_points" in plan_info:  # c = |det J|: the band Gauss points' c rides in the same launch
            work += 24 * (plan_info["coef_points"] - sz["q1"] * sz["q2"])
            per += " + 24 B per band Gauss point (its c and coordinates)"
        return ("hbm", work, per)
    if base == "k_cut_elem":
        return ("mfma", 2 * sz["n_cut_nodes"] * L * (L + 1) // 2,
                f"n_nodes L(L+1)/2 FMA = 2 x {L * (L + 1) // 2} flops per node")
    if base == "k_cut_elem_sides":  # DWQ: the side rules' systems run beside the cut element matrices
        return ("mfma", 2 * sz["n_cut_nodes"] * L * (L + 1) // 2,
                f"n_nodes L(L+1)/2 FMA = 2 x {L * (L + 1) // 2} flops per node (the cut element matrices); "
                "the DWQ side rules' refined systems run beside them in the same launch, uncounted")
    if base == "k_dwq_rows":
        return ("hbm", 8 * W2 * sz["n_dwq_rows"],
                f"8 (2p+1)^2 = {8 * W2} B per DWQ row: its box part, one value per slot")
    if base == "k_coef":  # a launch of its own (formations over resident tables): the WQ grid or the band points
        npts = plan_info.get("coef_points", sz["q1"] * sz["q2"])
        return ("hbm", (24 * npts + 16 * sz["n1"] * sz["n2"]) // 2,
                "24 B per point (c and its coordinates) + control points once, over the two launches")
    if base == "k_weights_coef":  # the weights and c = |det J| on the WQ grid in one launch
        return ("hbm", 24 * sz["q1"] * sz["q2"] + 16 * sz["n1"] * sz["n2"],
                "24 B per WQ-grid point (c and its coordinates) + control points once; the weight systems "
                "of Eq. (5) run beside them in the same launch")
    if base == "k_wq_weights":
        m, q = 2 * p + 1, 2 * p + 2
        return ("alu", (sz["n1"] + sz["n2"]) * (2 * q * m * m - (2 * m ** 3) // 3),
                f"Householder QR of {q}x{m}: 2qm^2 - 2m^3/3 flops per test function")
    if base == "k_cutprep":
        return ("hbm", 24 * sz["n_cut_nodes"], "24 B (x, y, w) per cut node written")
    if base == "k_cut_rows" and name.endswith(",cut>"):
        return ("hbm", 8 * L * L * sz["n_cut_el"] + 8 * W2 * plan_info.get("n_form_rows", sz["n_cut_fn"]),
                "8 L^2 B per cut element matrix read + 8 (2p+1)^2 B per element-formed row")
    if base == "k_cut_rows":
        fl = 2 * (L * (2 * p + 1) * (p + 1) + W2 * L)
        return ("alu", fl * plan_info.get("n_form_rows", sz["n_cut_fn"]),
                f"sum-factorised Gauss per row: 2((p+1)^3 (2p+1) + (2p+1)^2 (p+1)^2) = {fl} flops")
    return None


def kernel_breakdown(plan, step, steps, sz, peaks, plan_info, N=None):
    """Every kernel of the step with its mean time per step (per-kernel HIP events, kernel by kernel)."""
    plan.set_graph(False)
    plan.set_timing(True, per_kernel=True)
    for _ in range(2):
        step()
    plan.kernel_times()  # drop the warm-up
    for _ in range(steps):
        step()
    kt = plan.kernel_times()
    plan.set_timing(False)
    plan.set_graph(True)
    rows = []
    for name, (ms, cnt) in kt.items():
        rows.append({"kernel": name, "ms_per_step": ms / steps, "launches_per_step": cnt / steps,
                     "avg_launch_ms": ms / max(1, cnt)})
    rows.sort(key=lambda r: -r["ms_per_step"])
    roofs = {}
    for r in rows:
        w = kernel_work(r["kernel"], sz, plan_info)
        if w is not None:
            roofs[r["kernel"]] = _roof(r["kernel"], w[0], w[1], r["avg_launch_ms"], peaks, w[2],
                                       "HIP events at the dispatch's start and end, kernel by kernel on two streams",
                                       traffic=_traffic(r["kernel"], sz["p"], N) if N else None)
    return rows, roofs


# ---------------------------------------------------------------- CPU oracle
def _oracle_sample(args):
    """One process: the oracle set-up on the full patch, then its share of sampled rows."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.assemble import Oracle
    from paper_2101_08053_amd import workloads as wl
    N, p, sample_rows, seed = args
    with threadpool_limits(limits=1):
        cfg = wl.config2(N=N, p=p)
        t0 = time.perf_counter()
        o = Oracle(cfg)
        t_setup = time.perf_counter() - t0
        interior = o.interior_rows_flat()
        cut = o.cut_rows_flat()
        k_int = min(sample_rows, len(interior))
        frac = k_int / max(1, len(interior))
        k_cut = max(1, int(round(frac * len(cut))))
        rng = np.random.default_rng(seed)
        ri = np.sort(rng.choice(interior, k_int, replace=False))
        rc = np.sort(rng.choice(cut, k_cut, replace=False))
        t1 = time.perf_counter()
        Mi = o.wq_rows(ri)
        ts = o.ts
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
        return {"nnz": int(Mi.nnz + Mc.nnz), "t_rows": t_rows, "t_setup": t_setup, "frac": frac,
                "k_int": k_int, "k_cut": k_cut}


def _host():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(args):
    """The oracle (plain NumPy, as it stands) on bounded samples of the headline workload.

    Each process sets up the oracle on the full patch (trimming, weights),
    then forms `cpu_rows` sampled interior rows (weighted-quadrature double
    sums) and a proportional share of the cut rows (element Gauss + cut
    rule), each sample drawn with its own seed. Rate = sampled structural
    nonzeros over the time of the rows plus the set-up charged in proportion
    to the share of rows sampled. One process on one core, then one process
    per host core (at most 16) side by side: wall clock of the slowest.
    """
    import concurrent.futures as cf
    import multiprocessing as mp
    one = _oracle_sample((args.N, args.p, args.cpu_rows, 0))
    t1 = one["t_rows"] + one["frac"] * one["t_setup"]
    host = _host()
    procs = args.cpu_procs or min(16, host["nproc"] or 1)
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(procs, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_oracle_sample, [(args.N, args.p, args.cpu_rows, 1 + k) for k in range(procs)]))
    wall = time.perf_counter() - t0
    nnz = sum(r["nnz"] for r in res)
    t_rows = max(r["t_rows"] for r in res)
    t_setup = max(r["t_setup"] for r in res)
    frac = res[0]["frac"]
    t_all = t_rows + frac * t_setup
    return {"value": nnz / t_all, "unit": "nnz/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} processes (one thread each), each: oracle set-up on the full p={args.p} "
                      f"{args.N}^2 patch ({t_setup:.1f} s, charged x{frac:.3f}) + {res[0]['k_int']} interior rows + "
                      f"{res[0]['k_cut']} cut rows, its own seed ({nnz} nnz in {t_rows:.1f} s of rows; "
                      f"{wall:.1f} s wall)",
            "one_core": {"value": one["nnz"] / t1, "cores": 1,
                         "sample": f"{one['k_int']} interior + {one['k_cut']} cut rows, {one['nnz']} nnz in "
                                   f"{one['t_rows']:.1f} s + set-up {one['t_setup']:.1f} s charged x{one['frac']:.3f}"},
            "host": host}


# ---------------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the formation path runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2101_08053_amd import igatrim
    from paper_2101_08053_amd import workloads as wl

    if not os.path.exists(igatrim.LIB_PATH):
        from paper_2101_08053_amd import build
        build.build()
    # the oracle first, in processes forked before this one touches the GPU
    cpu = None if (args.no_cpu or args.copy_calibration) else cpu_baseline(args)
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
    peaks = igatrim.measure_peaks(1024, 5)
    print(f"# peaks {peaks}", file=sys.stderr, flush=True)
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
    print(f"# headline {ms_step:.4f} ms", file=sys.stderr, flush=True)
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
    # every kernel of the step with its own dispatch events
    plan_info = {"coef_points": sz["n_points"] - sz["n_cut_nodes"], "n_form_rows": sz["n_cut_fn"]}
    kernels, kroofs = kernel_breakdown(plan, step, args.steps, sz, peaks, plan_info, N=args.N)
    dominant = kernels[0]["kernel"]

    # interior rows alone (phase events: the kernel runs alone), HBM bound
    int_ms, int_cnt = phases["interior"]
    k_ms = int_ms / max(1, int_cnt)
    alg_bytes = 8 * sz["band"] * sz["n_interior"] + 8 * sz["q1"] * sz["q2"]
    traffic = _traffic(f"k_interior<{args.p}>", args.p, args.N)
    interior_alone = _roof(f"k_interior<{args.p}>", "hbm", alg_bytes, k_ms, peaks,
                           f"8 (2p+1)^2 B per interior row + 8 B per WQ point",
                           "HIP events at the dispatch's start and end, the kernel alone on the GPU (phase timing)",
                           traffic=traffic)
    roof = dict(kroofs.get(dominant) or {"kernel": dominant, "bound": None, "note": "no algorithmic work defined"})
    roof["ms_per_step"] = round(kernels[0]["ms_per_step"], 5)
    roof["chosen"] = "largest time per step among the step's kernels (per-kernel dispatch events)"

    # the step with the last-level cache flushed between replays: a 1 GiB write, then one replay
    # timed by events on the stream
    scratch = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cold = []
    for k in range(args.steps + 2):
        scratch.fill_(float(k))
        ev0.record(stream)
        step()
        ev1.record(stream)
        ev1.synchronize()
        if k >= 2:
            cold.append(ev0.elapsed_time(ev1))
    del scratch
    ms_cold = statistics.median(cold)

    out = {
        "metric": "mass-matrix nnz formed/s (FP64, p=4 trimmed 256^2)",
        "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"trimmed patch p={args.p}, {args.N}x{args.N} elements, perturbed geometry "
                               "c=|det J|, 16-point cubic B-spline hole, hybrid Gauss, whole formation path",
                   "p": args.p, "elements": [args.N, args.N], "n_act": sz["n_act"], "nnz": nnz,
                   "n_interior": sz["n_interior"], "n_cut_fn": sz["n_cut_fn"], "n_cut_el": sz["n_cut_el"],
                   "n_cut_nodes": sz["n_cut_nodes"], "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": None,
        "peaks_measured": peaks,
        "kernels": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()} for r in kernels],
        "rooflines": {"interior_alone": interior_alone, **kroofs},
        "launches": {"graph_ms_per_step": ms_step, "kernel_by_kernel_ms_per_step": ms_eager,
                     "with_phase_events_ms_per_step": ms_timed},
        # a phase's event pairs summed over the timed pass (a phase may run on both streams: the
        # pairs overlap, so the phases need not add up to the step)
        "phases_ms_per_step": {k: round(v[0] / args.steps, 5) for k, v in phases.items()},
        "formation_only": {"ms_per_step": ms_form, "value": nnz / (ms_form * 1e-3), "unit": "nnz/s",
                           "note": "tables resident; coefficient + interior rows + cut rows"},
        "cache_flushed": {"ms_per_step": ms_cold, "value": nnz / (ms_cold * 1e-3), "unit": "nnz/s",
                          "note": "median over replays, each after a 1 GiB write (events on the stream)"},
    }
    del vals
    if not args.no_extra:
        wanted = set(args.sections.split(","))
        for key, fn in (("dwq", bench_dwq), ("config3_dwq", bench_config3), ("projection", bench_projection),
                        ("batched", bench_batched), ("adjoint", bench_adjoint), ("table1", bench_table1)):
            if key not in wanted:
                continue
            out[key] = fn(igatrim, wl, cfg, args, sync, stream, peaks)
            print(f"# {key} done", file=sys.stderr, flush=True)
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_dwq(igatrim, wl, cfg, args, sync, stream, peaks):
    """The headline workload with discontinuous weighted quadrature for the cut rows."""
    import torch
    plan = igatrim.Plan(cfg, igatrim.DWQ)
    sz = plan.sizes
    coef = plan.coeff()
    vals = torch.empty((sz["band"], sz["n_act"]), dtype=torch.float64, device="cuda")
    ms_full = _timed(lambda: plan.mass_form(coef, out=vals, full=True, stream=stream), args.steps, args.warmup, sync)
    ms_form = _timed(lambda: plan.mass_form(coef, out=vals, stream=stream), args.steps, 2, sync)
    plan.status()
    steps = max(5, args.steps // 5)
    kernels, kroofs = kernel_breakdown(plan, lambda: plan.mass_form(coef, out=vals, full=True, stream=stream), steps,
                                       sz, peaks, {"coef_points": sz["n_points"] - sz["n_cut_nodes"]})
    sides = [r for r in kernels if r["kernel"].startswith(("k_dwq_sides", "k_cut_elem_sides"))]
    # the section's roofline: the kernel with the largest time per step among those with a work count
    top = next((r["kernel"] for r in kernels if r["kernel"] in kroofs), None)
    return {"value": sz["nnz"] / (ms_full * 1e-3), "unit": "nnz/s", "ms_per_step": ms_full,
            "formation_only_ms": ms_form, "formation_only_value": sz["nnz"] / (ms_form * 1e-3),
            "n_dwq_rows": sz["n_dwq_rows"], "n_cut_fn": sz["n_cut_fn"],
            "side_rules_ms_per_step": sides[0]["ms_per_step"] if sides else None,
            "side_rules_kernel": sides[0]["kernel"] if sides else None,
            "roofline": dict(kroofs[top], chosen="largest time per step among the step's counted kernels")
            if top else None,
            "rooflines": kroofs,
            "kernels": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()} for r in kernels[:8]],
            "note": "same workload and step as the headline, cut rows by DWQ boxes + element rules"}


def bench_config3(igatrim, wl, cfg, args, sync, stream, peaks):
    """Degree 6, 512^2 elements, union of three seeded ellipses, DWQ: the HBM-sized single patch."""
    import torch
    c3 = wl.config3(N=args.cfg3_N)
    t0 = time.perf_counter()
    plan = igatrim.Plan(c3, igatrim.DWQ)
    t_plan = time.perf_counter() - t0
    sz = plan.sizes
    coef = plan.coeff()
    vals = torch.empty((sz["band"], sz["n_act"]), dtype=torch.float64, device="cuda")
    steps = max(5, args.steps // 5)
    ms_full = _timed(lambda: plan.mass_form(coef, out=vals, full=True, stream=stream), steps, 3, sync)
    ms_form = _timed(lambda: plan.mass_form(coef, out=vals, stream=stream), steps, 2, sync)
    plan.status()
    kernels, kroofs = kernel_breakdown(plan, lambda: plan.mass_form(coef, out=vals, full=True, stream=stream), steps,
                                       sz, peaks, {"coef_points": sz["n_points"] - sz["n_cut_nodes"]})
    band_bytes = 8 * sz["band"] * sz["n_act"]
    sides = [r for r in kernels if r["kernel"].startswith(("k_dwq_sides", "k_cut_elem_sides"))]
    return {"value": sz["nnz"] / (ms_full * 1e-3), "unit": "nnz/s", "ms_per_step": ms_full,
            "formation_only_ms": ms_form, "formation_only_value": sz["nnz"] / (ms_form * 1e-3),
            "band_MB": band_bytes / 1e6, "formation_only_GBs_written": band_bytes / (ms_form * 1e-3) / 1e9,
            "nnz": sz["nnz"], "n_act": sz["n_act"], "n_cut_fn": sz["n_cut_fn"], "n_cut_el": sz["n_cut_el"],
            "n_dwq_rows": sz["n_dwq_rows"], "plan_setup_s": round(t_plan, 2),
            "side_rules_ms_per_step": sides[0]["ms_per_step"] if sides else None,
            "side_rules_kernel": sides[0]["kernel"] if sides else None,
            "kernels": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()} for r in kernels[:10]],
            "rooflines": {k: v for k, v in kroofs.items() if k.startswith(("k_interior", "k_cut_elem"))},
            "note": f"p=6, {args.cfg3_N}^2 elements, perturbed geometry c=|det J|, hole = union of 3 seeded "
                    "ellipses, DWQ; whole path (graph replay) and formation over resident tables"}


def bench_projection(igatrim, wl, cfg, args, sync, stream, peaks):
    """L2 projection (right-hand side + Jacobi PCG to 1e-12) on the headline workload's matrix."""
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
    # per iteration: the symmetrised band values (8 B) and their column table (4 B) once, and about seven
    # vectors
    bytes_it = 12 * sz["band"] * sz["n_act"] + 7 * 8 * sz["n_act"]
    roof = _roof("PCG iteration (k_cg_spmv_c, k_cg_update_c, k_cg_dir_c)", "hbm", bytes_it, ms / it, peaks,
                 "12 B per band slot (value + column) + 7 x 8 B per row",
                 "whole solve timed on the host (synchronous call) / iterations")
    # the same projection in the extended B-spline basis (outer functions tied to blocks of inner ones)
    igatrim.l2_project_ext(plan, vals, coef, g, rtol=1e-12)  # warm-up: workspace allocation
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        ue, info_e = igatrim.l2_project_ext(plan, vals, coef, g, rtol=1e-12)
    sync()
    ms_e = 1e3 * (time.perf_counter() - t0) / reps
    ext = {"ms": ms_e, "iterations": info_e["iterations"], "rel_residual": info_e["rel_residual"],
           "ms_per_iteration": ms_e / max(1, info_e["iterations"]),
           "max_abs_coefficient": float(ue.abs().max()), "max_abs_coefficient_plain": float(u.abs().max()),
           "note": "extension built from the classes in every call; per iteration the band product of E^T p, "
                   "the update (forming E A E^T p row by row) and the direction (forming E^T of it); "
                   "functions cut to slivers take huge coefficients in the plain basis, not in the extended one"}
    return {"ms": ms, "iterations": info["iterations"], "rel_residual": info["rel_residual"],
            "ms_per_iteration": ms / it, "roofline": roof, "extended": ext,
            "note": "target g = sin(2x) cos(3y), c = |det J|; rhs + symmetrisation + Jacobi PCG, synchronous"}


def bench_batched(igatrim, wl, cfg_unused, args, sync, stream, peaks):
    """256 patches (p 2..5, 16..256 elements per direction, one ellipse each): batched vs one by one,
    formed and L2-projected."""
    import torch
    cfgs = wl.config4(n_patch=args.batch)
    t0 = time.perf_counter()
    plans = [igatrim.Plan(c, igatrim.HYBRID_GAUSS) for c in cfgs]
    t_plan = time.perf_counter() - t0
    coeffs = [p.coeff() for p in plans]
    nnz = sum(p.sizes["nnz"] for p in plans)
    band_bytes = sum(8 * p.sizes["band"] * p.sizes["n_act"] for p in plans)
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
    # the batched L2 projection of all patches (g = sin(pi x) cos(pi y) at physical points)
    g = igatrim.target_sincos(math.pi, 0.0, math.pi, 0.0)
    b.form(use_graph=True)
    b.project([g] * len(plans), rtol=1e-12)  # first call: buffers
    sync()
    t0 = time.perf_counter()
    us, infos = b.project([g] * len(plans), rtol=1e-12)
    sync()
    ms_proj = 1e3 * (time.perf_counter() - t0)
    iters = [i["iterations"] for i in infos]
    # the same projections one patch at a time
    t0 = time.perf_counter()
    for p, c, o in zip(plans, coeffs, outs):
        igatrim.l2_project(p, o, c, g, rtol=1e-12)
    sync()
    ms_proj_plain = 1e3 * (time.perf_counter() - t0)
    roof = _roof("batched formation (graph replay)", "hbm", band_bytes, ms_graph, peaks,
                 "8 B per band value written (all patches)", "whole replay timed on the host / replays")
    # the same patches with the degree-5 ones formed by DWQ (their side rules solved in the batch too)
    plans5 = [igatrim.Plan(c, igatrim.DWQ) if c.p == 5 else p for c, p in zip(cfgs, plans)]
    coeffs5 = [p.coeff() for p in plans5]
    b5 = igatrim.Batch(plans5, coeffs5)
    b5.autotune()
    ms_dwq5 = _timed(lambda: b5.form(use_graph=True), steps, 2, sync)
    b5.status()
    outs5 = b5.outs

    def plain5():
        for p, c, o in zip(plans5, coeffs5, outs5):
            p.mass_form(c, out=o)

    ms_dwq5_plain = _timed(plain5, max(3, steps // 2), 2, sync)
    n_dwq5 = sum(1 for c in cfgs if c.p == 5)
    nnz5 = sum(p.sizes["nnz"] for p in plans5)
    del b5, outs5
    return {"value": nnz / (ms_graph * 1e-3), "unit": "nnz/s", "ms": ms_graph, "eager_ms": ms_eager,
            "plain_ms": ms_plain, "plain_value": nnz / (ms_plain * 1e-3), "speedup_vs_plain": ms_plain / ms_graph,
            "patches": len(plans), "nnz": nnz, "band_MB": band_bytes / 1e6, "roofline": roof,
            "items": info["n_items"], "grid": info["grid"],
            "wg_per_cu": info["wg_per_cu"], "chunk": info["chunk"],
            "cut_elements": "persistent queue" if info["grid"] > 0 else "one workgroup each (autotuner's choice)",
            "autotune_best_ms": tune_ms, "plan_setup_s": round(t_plan, 2),
            "projection_ms": ms_proj, "projection_plain_ms": ms_proj_plain,
            "projection_speedup_vs_plain": ms_proj_plain / ms_proj,
            "projection_iterations": {"max": max(iters), "median": statistics.median(iters), "sum": sum(iters)},
            "projection_converged": all(i["converged"] for i in infos),
            "dwq_p5": {"ms": ms_dwq5, "value": nnz5 / (ms_dwq5 * 1e-3), "plain_ms": ms_dwq5_plain,
                       "speedup_vs_plain": ms_dwq5_plain / ms_dwq5, "dwq_patches": n_dwq5,
                       "note": "the same 256 patches with the degree-5 ones by DWQ: their side rules (refined "
                               "minimum-norm solves) batched across patches in the replay, then their box rows; "
                               "the one-by-one calls form over the plans' resident side rules (no solves)"},
            "note": "formation over resident tables, one graph replay per call (cut element matrices beside "
                    "per-degree coefficient and interior launches, then the element-formed rows) vs one formation "
                    "call per patch; projection: batched right-hand sides + PCG of all patches (synchronous) vs "
                    "one projection call per patch"}


def bench_adjoint(igatrim, wl, cfg_unused, args, sync, stream, peaks):
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
    y = torch.empty_like(u)
    ms_fwd_na = _timed(lambda: igatrim.mf_apply_noalloc(plan, c, u, y), steps, 2, sync)
    coef = plan.coeff(igatrim.COEF_AT_POINTS, c_points=c)
    vals = torch.empty((sz["band"], sz["n_act"]), dtype=torch.float64, device="cuda")
    ms_form = _timed(lambda: plan.mass_form(coef, out=vals), steps, 2, sync)
    nnz = sz["nnz"]
    n, npts = sz["n_act"], sz["n_points"]
    # algorithmic bytes: forward reads u and c, writes y; adjoint reads u, c, r, writes du and dc
    fwd_bytes = 8 * (2 * n + npts)
    bwd_bytes = 8 * (3 * n + 2 * npts)
    # the one-launch kernels alone (per-kernel HIP events)
    plan.set_timing(True, per_kernel=True)
    for _ in range(2):
        igatrim.mf_apply(plan, c, u)
        igatrim.mf_adjoint(plan, c, u, gy)
    plan.kernel_times()
    for _ in range(steps):
        igatrim.mf_apply(plan, c, u)
        igatrim.mf_adjoint(plan, c, u, gy)
    kt = plan.kernel_times()
    plan.set_timing(False)
    p = sz["p"]
    nq = sz["q1"] * sz["q2"]
    kernels = {k: {"avg_launch_ms": ms / max(1, cnt), "calls": cnt} for k, (ms, cnt) in kt.items()}
    grid_roofs = {}
    # the one-launch kernels: the grid part and the element vectors (Ue, (p+1)^2 entries per band or cut
    # element) beside it
    ue = (p + 1) ** 2 * (sz["n_band_el"] + sz["n_cut_el"])
    for name, nbytes, per in ((f"k_mf_fwd<{p}>", 8 * (npts + 2 * n + ue),
                               "8 B per rule-point c, per u, y value and per element-vector entry written"),
                              (f"k_mf_adj<{p}>", 8 * (2 * npts + 3 * n + ue),
                               "8 B per rule-point c, dc, per u, r, du value and per element-vector entry written")):
        if name in kernels:
            grid_roofs[name] = _roof(name, "hbm", nbytes, kernels[name]["avg_launch_ms"], peaks, per,
                                     "HIP events at the dispatch's start and end",
                                     traffic=_traffic(name, p, args.mf_N))
    return {"forward_ms": ms_fwd, "backward_ms": ms_bwd, "forward_noalloc_ms": ms_fwd_na,
            "plain_formation_ms": ms_form,
            "forward_value": nnz / (ms_fwd * 1e-3), "backward_value": nnz / (ms_bwd * 1e-3),
            "plain_value": nnz / (ms_form * 1e-3), "unit": "nnz-equivalent/s", "nnz": nnz,
            "n_act": n, "n_points": npts,
            "rooflines": {
                "forward": _roof("matrix-free forward (k_mf_fwd, k_mf_rows)",
                                 "hbm", fwd_bytes, ms_fwd, peaks, "8 B per u, y value and per rule-point c",
                                 "whole call timed on the host / calls"),
                "adjoint": _roof("matrix-free adjoint (k_mf_adj, k_mf_fix, k_mf_gather_add)",
                                 "hbm", bwd_bytes, ms_bwd, peaks, "8 B per u, r, du value and per rule-point c, dc",
                                 "whole call timed on the host / calls"),
                **grid_roofs},
            "kernels": kernels,
            "note": f"p=4, {args.mf_N}^2 elements, c at every rule point; y = M(c)u and (dL/du, dL/dc)"}


def bench_table1(igatrim, wl, cfg_unused, args, sync, stream, peaks):
    """Table 1 (Sect. 4.1) from the device: each method's deviation from element Gauss, line trim, c = 1."""
    from paper_2101_08053_amd import experiments
    res = experiments.table1(degrees=tuple(range(1, 9)))
    return {"frobenius": {str(p): {c: r[c][0] for c in experiments.METHOD_COLUMNS} for p, r in res.items()},
            "spectral": {str(p): {c: r[c][1] for c in experiments.METHOD_COLUMNS} for p, r in res.items()},
            "paper": {str(p): dict(zip(experiments.METHOD_COLUMNS, v)) for p, v in experiments.PAPER_TABLE1.items()},
            "markdown": experiments.table1_markdown(res),
            "note": "line trim 10x10 elements, c = 1; ||M_method - M_gauss|| with every matrix formed on the device; "
                    "the paper's line is only drawn, so a seeded line stands in (magnitudes comparable)"}


if __name__ == "__main__":
    main()
