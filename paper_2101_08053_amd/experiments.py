"""The accuracy experiment of Sect. 4.1 (Table 1) run on the device.

On the line trim (10 x 10 elements, c = 1) the mass matrix is formed on the
GPU by element-wise Gauss (the reference), hybrid Gauss, discontinuous
weighted quadrature and naive weighted quadrature (c := 0 in the hole), and
each fast method's deviation from the reference is reported in the Frobenius
norm (absolute; the paper's "Euclidean norm" read as the norm of the
difference's entries) and in the spectral norm. Every matrix comes from the
library's kernels; this module only converts the band layout to a dense
matrix and takes norms.
"""
from __future__ import annotations

import numpy as np

# Sect. 4.1, Table 1: hybrid Gauss, discontinuous WQ, naive WQ (p = 1..6)
PAPER_TABLE1 = {
    1: (4.68883379e-17, 4.69071638e-17, 3.33078900e-03),
    2: (2.18894391e-17, 2.19723138e-17, 3.38923479e-04),
    3: (4.98024622e-17, 4.98024919e-17, 3.03838755e-04),
    4: (3.80411220e-16, 3.84739261e-16, 1.78250728e-04),
    5: (1.01851172e-15, 1.01851512e-15, 1.59974261e-04),
    6: (2.00575179e-15, 2.00590425e-15, 1.28293909e-04),
}
METHOD_COLUMNS = ("hybrid_gauss", "dwq", "naive_wq")


def band_to_dense(vals, fn_of, act_of, n1, n2, p):
    """Dense n_act x n_act matrix from the slot-major band layout (slot s = (a+p)(2p+1) + (b+p))."""
    W = 2 * p + 1
    n = vals.shape[1]
    D = np.zeros((n, n))
    f = np.asarray(fn_of, dtype=np.int64)
    i1, i2 = f % n1, f // n1
    for s in range(W * W):
        a, b = s // W - p, s % W - p
        j1, j2 = i1 + a, i2 + b
        ok = (j1 >= 0) & (j1 < n1) & (j2 >= 0) & (j2 < n2)
        col = np.full(n, -1, dtype=np.int64)
        col[ok] = act_of[(j2[ok] * n1 + j1[ok])]
        m = col >= 0
        D[np.nonzero(m)[0], col[m]] = vals[s, m]
    return D


def table1(degrees=(1, 2, 3, 4, 5, 6), N=10):
    """{p: {column: (frobenius, spectral)}} of each method's deviation from element Gauss, on the device."""
    from . import igatrim
    from . import workloads as wl
    methods = {"reference": igatrim.GAUSS_REF, "hybrid_gauss": igatrim.HYBRID_GAUSS, "dwq": igatrim.DWQ,
               "naive_wq": igatrim.NAIVE_WQ}
    out = {}
    for p in degrees:
        cfg = wl.table1_line(p, N=N)
        dense = {}
        for name, m in methods.items():
            plan = igatrim.Plan(cfg, m)
            vals = plan.mass_form(plan.coeff(igatrim.COEF_CONST, 1.0), full=True).cpu().numpy()
            plan.status()
            act_of, fn_of, _ = plan.index_maps()
            sz = plan.sizes
            dense[name] = band_to_dense(vals, fn_of.cpu().numpy(), act_of.cpu().numpy(), sz["n1"], sz["n2"], p)
            plan.close()
        ref = dense["reference"]
        out[p] = {c: (float(np.linalg.norm(dense[c] - ref)), float(np.linalg.norm(dense[c] - ref, 2)))
                  for c in METHOD_COLUMNS}
    return out


def table1_markdown(res):
    """The device's table beside the paper's columns (paper values for p <= 6)."""
    lines = ["| p | hybrid Gauss (device) | paper | DWQ (device) | paper | naive WQ (device) | paper | "
             "spectral: hybrid / DWQ / naive (device) |",
             "|---|---|---|---|---|---|---|---|"]
    for p, r in sorted(res.items()):
        pap = PAPER_TABLE1.get(p, (None, None, None))
        cells = [f"{p}"]
        for k, c in enumerate(METHOD_COLUMNS):
            cells.append(f"{r[c][0]:.3e}")
            cells.append(f"{pap[k]:.3e}" if pap[k] is not None else "-")
        cells.append(" / ".join(f"{r[c][1]:.2e}" for c in METHOD_COLUMNS))
        lines.append("| " + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"
