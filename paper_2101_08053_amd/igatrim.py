"""Python binding of libigatrim.so (ctypes): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module
turns Python/NumPy inputs into the C structs of ``include/iga_trim.h``,
allocates outputs as torch tensors on the current HIP device and passes
torch's current stream. It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IGA_TRIM_LIB names another build of the library (the index-checking test build)
LIB_PATH = os.environ.get("IGA_TRIM_LIB") or os.path.join(HERE, "libigatrim.so")

GAUSS_REF, HYBRID_GAUSS, DWQ, NAIVE_WQ = 0, 1, 2, 3
COEF_CONST, COEF_GEOM_DETJ, COEF_AT_POINTS = 0, 1, 2
FORM_FULL = 1
TARGET_SINCOS, TARGET_MONOMIAL, TARGET_AT_POINTS = 0, 1, 2
PHASES = ("setup", "coef", "interior", "cut")

STATUS = {0: "IGA_OK", -1: "IGA_E_INVALID", -2: "IGA_E_UNSUPPORTED", -3: "IGA_E_NOMEM", -4: "IGA_E_HIP",
          -5: "IGA_E_SINGULAR_WEIGHTS", -6: "IGA_E_TOPOLOGY", -7: "IGA_E_CAPACITY", -8: "IGA_E_NOCONV"}


class IgaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class iga_curve(C.Structure):
    _fields_ = [("kind", C.c_int32), ("degree", C.c_int32), ("n_cp", C.c_int32), ("reserved", C.c_int32),
                ("cp", C.POINTER(C.c_double)), ("cx", C.c_double), ("cy", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("phi", C.c_double)]


class iga_patch_desc(C.Structure):
    _fields_ = [("degree", C.c_int32), ("method", C.c_int32), ("n_knots", C.c_int32 * 2),
                ("knots", C.POINTER(C.c_double) * 2), ("n_curves", C.c_int32), ("reserved", C.c_int32),
                ("curves", C.POINTER(iga_curve))]


class iga_opts(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_q", C.c_int32), ("n_s", C.c_int32), ("reserved", C.c_int32 * 5)]


_SIZE_FIELDS = ["p", "N1", "N2", "n1", "n2", "n_act", "n_interior", "n_cut_fn", "n_cut_el", "n_band_el", "band",
                "q1", "q2", "n_cut_nodes", "n_points", "nnz", "n_arcs", "n_dwq_rows", "workspace_bytes"]


class iga_sizes(C.Structure):
    _fields_ = [(f, C.c_int64) for f in _SIZE_FIELDS]


class iga_coeff(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("value", C.c_double),
                ("geom_cp", C.c_void_p), ("c_points", C.c_void_p)]


class iga_target(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("w", C.c_double * 4), ("g_points", C.c_void_p)]


class iga_batch_stats(C.Structure):
    _fields_ = [("n_plans", C.c_int64), ("n_items", C.c_int64), ("nnz", C.c_int64), ("grid", C.c_int32),
                ("wg_per_cu", C.c_int32), ("order", C.c_int32), ("graph_ready", C.c_int32),
                ("chunk", C.c_int32), ("capped", C.c_int32)]


class iga_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("ms", C.c_double), ("count", C.c_int64)]


class iga_peaks(C.Structure):
    _fields_ = [("copy_gbs", C.c_double), ("fma_tflops", C.c_double), ("mfma_f64_tflops", C.c_double),
                ("n_cu", C.c_int32), ("reserved", C.c_int32)]


class iga_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double)]


_lib = None


def lib():
    """Load libigatrim.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch has loaded
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_08053_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, V = C.c_void_p, C.c_void_p
        sig = {
            "iga_trim_plan_create": (C.c_int, [C.POINTER(iga_patch_desc), C.POINTER(iga_opts), C.POINTER(P)]),
            "iga_plan_destroy": (None, [P]),
            "iga_plan_sizes": (C.c_int, [P, C.POINTER(iga_sizes)]),
            "iga_plan_points": (C.c_int, [P, C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]),
            "iga_plan_index_maps": (C.c_int, [P, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
            "iga_trim_mass_form": (C.c_int, [P, C.POINTER(iga_coeff), V, C.c_int32, V]),
            "iga_status_get": (C.c_int, [P, V]),
            "iga_trim_l2_project": (C.c_int, [P, C.POINTER(iga_coeff), V, C.POINTER(iga_target), C.c_double,
                                              C.c_int32, V, C.POINTER(iga_solve_info), V]),
            "iga_trim_rhs": (C.c_int, [P, C.POINTER(iga_coeff), C.POINTER(iga_target), V, V]),
            "iga_trim_l2_project_ext": (C.c_int, [P, C.POINTER(iga_coeff), V, C.POINTER(iga_target), C.c_double,
                                                  C.c_int32, V, C.POINTER(iga_solve_info), V]),
            "iga_trim_extension": (C.c_int, [P, V, V, V]),
            "iga_mf_apply": (C.c_int, [P, V, V, V, V]),
            "iga_mf_apply_noalloc": (C.c_int, [P, V, V, V, V]),
            "iga_mf_adjoint": (C.c_int, [P, V, V, V, V, V, V]),
            "iga_trim_mass_form_batched": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(iga_coeff),
                                                     C.POINTER(C.c_void_p), C.c_int32, V]),
            "iga_batch_create": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(iga_coeff), C.POINTER(C.c_void_p),
                                           C.POINTER(P)]),
            "iga_batch_destroy": (None, [P]),
            "iga_batch_form": (C.c_int, [P, C.c_int32, V]),
            "iga_batch_autotune": (C.c_int, [P, V, C.POINTER(C.c_float)]),
            "iga_batch_info": (C.c_int, [P, C.POINTER(iga_batch_stats)]),
            "iga_batch_status": (C.c_int, [P, V]),
            "iga_batch_project": (C.c_int, [P, C.POINTER(iga_target), C.c_double, C.c_int32, C.POINTER(C.c_void_p),
                                            C.POINTER(iga_solve_info), V]),
            "iga_plan_set_timing": (C.c_int, [P, C.c_int32]),
            "iga_plan_set_graph": (C.c_int, [P, C.c_int32]),
            "iga_plan_timings": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
            "iga_plan_kernel_times": (C.c_int, [P, C.POINTER(iga_kernel_time), C.c_int32, C.POINTER(C.c_int32)]),
            "iga_copy": (C.c_int, [V, V, C.c_int64, V]),
            "iga_measure_peaks": (C.c_int, [V, V, C.c_int64, C.c_int32, C.POINTER(iga_peaks), V]),
            "iga_plan_table": (C.c_int, [P, C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]),
            "iga_plan_int_table": (C.c_int, [P, C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                             C.POINTER(C.c_int64)]),
            "iga_plan_set_weights": (C.c_int, [P, C.c_int32, V, V]),
            "iga_plan_set_dwq_weights": (C.c_int, [P, C.c_int32, V, V]),
            "iga_plan_set_cut_nodes": (C.c_int, [P, V, V, V, C.c_int64, V]),
            "iga_debug_bounds_hits": (C.c_int, [C.POINTER(C.c_int64), C.c_int32]),
            "iga_status_string": (C.c_char_p, [C.c_int]),
            "iga_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


EXPORTED = ("iga_trim_plan_create", "iga_plan_destroy", "iga_plan_sizes", "iga_plan_points", "iga_plan_index_maps",
            "iga_trim_mass_form", "iga_status_get", "iga_trim_l2_project", "iga_trim_rhs", "iga_mf_apply",
            "iga_trim_l2_project_ext", "iga_trim_extension", "iga_mf_apply_noalloc",
            "iga_mf_adjoint", "iga_trim_mass_form_batched", "iga_batch_create", "iga_batch_destroy",
            "iga_batch_form", "iga_batch_autotune", "iga_batch_info", "iga_batch_status", "iga_batch_project",
            "iga_plan_set_timing", "iga_plan_timings", "iga_plan_kernel_times", "iga_plan_set_graph",
            "iga_copy", "iga_measure_peaks", "iga_plan_table", "iga_plan_int_table", "iga_plan_set_weights",
            "iga_plan_set_dwq_weights", "iga_plan_set_cut_nodes", "iga_debug_bounds_hits", "iga_status_string",
            "iga_last_error")

(TABLE_WQ_POINTS, TABLE_WQ_WEIGHTS, TABLE_MASS_1D, TABLE_C_WQ, TABLE_C_BAND, TABLE_C_CUT, TABLE_CUT_W,
 TABLE_DWQ_X, TABLE_DWQ_W) = range(9)
ITABLE_DWQ_NPTS, ITABLE_DWQ_ELEM, ITABLE_DWQ_WQIDX, ITABLE_DWQ_BOX, ITABLE_FORM_ROWS = range(5)


def debug_bounds_hits(reset=False):
    """Out-of-range band stores counted by an index-checking build (IGA_TRIM_LIB); raises on a release build."""
    n = C.c_int64(0)
    _check(lib().iga_debug_bounds_hits(C.byref(n), 1 if reset else 0))
    return int(n.value)


def _check(code):
    if code != 0:
        raise IgaError(code, lib().iga_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the library runs on gfx950 GPUs only")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Plan:
    """A trimmed patch prepared on the device (iga_trim_plan_create)."""

    def __init__(self, patch, method=HYBRID_GAUSS, n_r=0, n_q=0, n_s=0):
        L = lib()
        self._keep = []
        desc = iga_patch_desc()
        desc.degree = patch.p
        desc.method = method
        for d in range(2):
            k = np.ascontiguousarray(patch.knots[d], dtype=np.float64)
            self._keep.append(k)
            desc.n_knots[d] = len(k)
            desc.knots[d] = k.ctypes.data_as(C.POINTER(C.c_double))
        curves = (iga_curve * max(1, len(patch.curves)))()
        for i, cv in enumerate(patch.curves):
            curves[i].kind = cv.kind
            curves[i].degree = cv.degree
            if cv.cp is not None:
                cp = np.ascontiguousarray(cv.cp, dtype=np.float64)
                self._keep.append(cp)
                curves[i].n_cp = len(cp)
                curves[i].cp = cp.ctypes.data_as(C.POINTER(C.c_double))
            curves[i].cx, curves[i].cy, curves[i].a, curves[i].b, curves[i].phi = cv.cx, cv.cy, cv.a, cv.b, cv.phi
        desc.n_curves = len(patch.curves)
        desc.curves = C.cast(curves, C.POINTER(iga_curve))
        opts = iga_opts(n_r, n_q, n_s)
        h = C.c_void_p()
        _torch()
        _check(L.iga_trim_plan_create(C.byref(desc), C.byref(opts), C.byref(h)))
        self.h = h
        self.patch = patch
        self.method = method
        s = iga_sizes()
        _check(L.iga_plan_sizes(h, C.byref(s)))
        self.sizes = {f: int(getattr(s, f)) for f in _SIZE_FIELDS}

    def close(self):
        if getattr(self, "h", None):
            lib().iga_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ views
    def _copy_dev(self, ptr, n, dtype):
        torch = _torch()
        out = torch.empty(n, dtype=dtype, device="cuda")
        if n:
            _check(lib().iga_copy(_dptr(out), ptr, n * out.element_size(), _stream()))
        return out

    def points(self):
        """(n_points, 2) parameter coordinates of every rule point (device copy)."""
        torch = _torch()
        xy = C.c_void_p()
        n = C.c_int64()
        _check(lib().iga_plan_points(self.h, C.byref(xy), C.byref(n)))
        return self._copy_dev(xy, 2 * n.value, torch.float64).view(-1, 2)

    def index_maps(self):
        torch = _torch()
        a, f, c = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(lib().iga_plan_index_maps(self.h, C.byref(a), C.byref(f), C.byref(c)))
        nf = self.sizes["n1"] * self.sizes["n2"]
        return (self._copy_dev(a, nf, torch.int32), self._copy_dev(f, self.sizes["n_act"], torch.int32),
                self._copy_dev(c, nf, torch.int8))

    def table(self, which, d=0):
        """Device copy of a plan table, reshaped (rows, stride)."""
        torch = _torch()
        ptr, n, st = C.c_void_p(), C.c_int64(), C.c_int64()
        _check(lib().iga_plan_table(self.h, which, d, C.byref(ptr), C.byref(n), C.byref(st)))
        return self._copy_dev(ptr, n.value, torch.float64).view(-1, st.value)

    def int_table(self, which, d=0):
        """Device copy of an integer plan table, reshaped (rows, stride)."""
        torch = _torch()
        ptr, n, st = C.c_void_p(), C.c_int64(), C.c_int64()
        _check(lib().iga_plan_int_table(self.h, which, d, C.byref(ptr), C.byref(n), C.byref(st)))
        return self._copy_dev(ptr, n.value, torch.int32).view(-1, st.value)

    def set_weights(self, d, W):
        """Inject weights of direction d (device tensor in the weight-table layout)."""
        _check(lib().iga_plan_set_weights(self.h, d, _dptr(W), _stream()))

    def set_dwq_weights(self, d, w):
        """Inject discontinuous weights of direction d (device tensor in the IGA_TABLE_DWQ_W layout)."""
        _check(lib().iga_plan_set_dwq_weights(self.h, d, _dptr(w), _stream()))

    def set_cut_nodes(self, x, y, w):
        """Inject cut-element nodes (device tensors of n_cut_nodes values)."""
        _check(lib().iga_plan_set_cut_nodes(self.h, _dptr(x), _dptr(y), _dptr(w), x.numel(), _stream()))

    # ---------------------------------------------------------- calls
    def coeff(self, kind=None, value=1.0, geom_cp=None, c_points=None):
        c = iga_coeff()
        c.kind = self.patch.coef if kind is None else kind
        c.value = value
        if c.kind == COEF_GEOM_DETJ:
            if geom_cp is None:
                geom_cp = self.geom_tensor()
            self._geom = geom_cp
            c.geom_cp = geom_cp.data_ptr()
        if c.kind == COEF_AT_POINTS:
            if c_points is None:
                raise ValueError("per-point coefficient needs c_points")
            self._cpts = c_points
            c.c_points = c_points.data_ptr()
        return c

    def geom_tensor(self):
        torch = _torch()
        if getattr(self, "_geom_t", None) is None:
            self._geom_t = torch.as_tensor(np.ascontiguousarray(self.patch.geom_cp), dtype=torch.float64,
                                           device="cuda")
        return self._geom_t

    def mass_form(self, coeff=None, out=None, full=False, stream=None):
        """Band values (band, n_act) of the mass matrix, slot-major."""
        torch = _torch()
        if coeff is None:
            coeff = self.coeff()
        if out is None:
            out = torch.empty((self.sizes["band"], self.sizes["n_act"]), dtype=torch.float64, device="cuda")
        _check(lib().iga_trim_mass_form(self.h, C.byref(coeff), _dptr(out), FORM_FULL if full else 0,
                                        _stream(stream)))
        return out

    def status(self, stream=None):
        _check(lib().iga_status_get(self.h, _stream(stream)))

    def set_timing(self, on=True, per_kernel=False):
        """Phase timing (on), per-kernel dispatch timing (per_kernel) or off."""
        _check(lib().iga_plan_set_timing(self.h, (2 if per_kernel else 1) if on else 0))

    def kernel_times(self):
        """{kernel name: (summed ms, dispatches)} since the last call (per-kernel timing)."""
        cap = 64
        buf = (iga_kernel_time * cap)()
        n = C.c_int32()
        _check(lib().iga_plan_kernel_times(self.h, buf, cap, C.byref(n)))
        return {buf[k].name.decode(): (buf[k].ms, int(buf[k].count)) for k in range(min(n.value, cap))}

    def set_graph(self, on=True):
        _check(lib().iga_plan_set_graph(self.h, 1 if on else 0))

    def timings(self):
        ms = (C.c_double * 4)()
        cnt = (C.c_int64 * 4)()
        _check(lib().iga_plan_timings(self.h, ms, cnt))
        return {PHASES[k]: (ms[k], int(cnt[k])) for k in range(4)}


def mass_form(patch, method=HYBRID_GAUSS, coef=None, **kw):
    """One-call form of the formation entry point: knots, degree, trim curves, c, method -> band values."""
    plan = Plan(patch, method, **kw)
    c = plan.coeff() if coef is None else coef
    return plan, plan.mass_form(c)


def _target(kind=TARGET_SINCOS, w=(math.pi, 0.0, math.pi, 0.0), g_points=None):
    t = iga_target()
    t.kind = kind
    for k in range(4):
        t.w[k] = w[k]
    t.g_points = g_points.data_ptr() if g_points is not None else None
    return t


def target_sincos(w0, w1, w2, w3):
    """g = sin(w0 x + w1) cos(w2 y + w3) at physical points."""
    return _target(TARGET_SINCOS, (w0, w1, w2, w3))


def target_monomial(e0, e1):
    """g = x^e0 y^e1 at physical points."""
    return _target(TARGET_MONOMIAL, (float(e0), float(e1), 0.0, 0.0))


def target_points(g_points):
    return _target(TARGET_AT_POINTS, (0, 0, 0, 0), g_points)


def rhs(plan, coeff, target, stream=None):
    torch = _torch()
    b = torch.empty(plan.sizes["n_act"], dtype=torch.float64, device="cuda")
    _check(lib().iga_trim_rhs(plan.h, C.byref(coeff), C.byref(target), _dptr(b), _stream(stream)))
    return b


def l2_project(plan, vals, coeff, target, rtol=1e-12, maxit=None, u0=None, stream=None, raise_on_noconv=True):
    """L2 projection (Sect. 4.2) with the plan's rules; returns (u, info dict)."""
    torch = _torch()
    n = plan.sizes["n_act"]
    u = torch.zeros(n, dtype=torch.float64, device="cuda") if u0 is None else u0.clone()
    info = iga_solve_info()
    maxit = maxit or 10 * n
    code = lib().iga_trim_l2_project(plan.h, C.byref(coeff), _dptr(vals), C.byref(target), rtol, maxit, _dptr(u),
                                     C.byref(info), _stream(stream))
    out = {"iterations": info.iterations, "converged": bool(info.converged), "rel_residual": info.rel_residual}
    if code != 0 and not (code == -8 and not raise_on_noconv):
        _check(code)
    return u, out


def l2_project_ext(plan, vals, coeff, target, rtol=1e-12, maxit=None, u0=None, stream=None, raise_on_noconv=True):
    """L2 projection in the extended B-spline basis (Sects. 2.2, 4.2); returns (u, info dict)."""
    torch = _torch()
    n = plan.sizes["n_act"]
    u = torch.zeros(n, dtype=torch.float64, device="cuda") if u0 is None else u0.clone()
    info = iga_solve_info()
    maxit = maxit or 10 * n
    code = lib().iga_trim_l2_project_ext(plan.h, C.byref(coeff), _dptr(vals), C.byref(target), rtol, maxit,
                                         _dptr(u), C.byref(info), _stream(stream))
    out = {"iterations": info.iterations, "converged": bool(info.converged), "rel_residual": info.rel_residual}
    if code != 0 and not (code == -8 and not raise_on_noconv):
        _check(code)
    return u, out


def extension(plan, stream=None):
    """Columns of the extension: (members, weights), each [n_act, (p+1)^2] on the device."""
    torch = _torch()
    n, L = plan.sizes["n_act"], (plan.patch.p + 1) ** 2
    members = torch.empty((n, L), dtype=torch.int32, device="cuda")
    weights = torch.empty((n, L), dtype=torch.float64, device="cuda")
    _check(lib().iga_trim_extension(plan.h, _dptr(members), _dptr(weights), _stream(stream)))
    return members, weights


def mf_apply(plan, c_points, u, stream=None):
    torch = _torch()
    y = torch.empty_like(u)
    _check(lib().iga_mf_apply(plan.h, _dptr(c_points), _dptr(u), _dptr(y), _stream(stream)))
    return y


def mf_apply_noalloc(plan, c_points, u, y, stream=None):
    """y = M(c) u into the caller's y with the library's static scratch (no device allocation)."""
    _check(lib().iga_mf_apply_noalloc(plan.h, _dptr(c_points), _dptr(u), _dptr(y), _stream(stream)))
    return y


def mf_adjoint(plan, c_points, u, gy, stream=None):
    torch = _torch()
    du = torch.empty_like(u)
    dc = torch.empty_like(c_points)
    _check(lib().iga_mf_adjoint(plan.h, _dptr(c_points), _dptr(u), _dptr(gy), _dptr(du), _dptr(dc),
                                _stream(stream)))
    return du, dc


def measure_peaks(mib=1024, reps=5, stream=None):
    """Measured copy bandwidth (GB/s) and FP64 FMA / matrix-core rates (TFLOP/s) of the current device."""
    torch = _torch()
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    pk = iga_peaks()
    _check(lib().iga_measure_peaks(_dptr(src), _dptr(dst), n, reps, C.byref(pk), _stream(stream)))
    return {"copy_GBs": pk.copy_gbs, "fma_f64_TFs": pk.fma_tflops, "mfma_f64_TFs": pk.mfma_f64_tflops,
            "compute_units": pk.n_cu, "copy_bytes_each_way": n * 8}


def _make_mass_apply():
    import torch

    class MassApply(torch.autograd.Function):
        """y = M(c) u through the library; backward calls the hand-written adjoint.

        Inputs: u (n_act) and c at every rule point (n_points), float64 on the
        device. Basis values are recomputed in the kernels, nothing per row is
        saved but u and c.
        """

        @staticmethod
        def forward(ctx, u, c_points, plan):
            u = u.contiguous()
            c_points = c_points.contiguous()
            ctx.plan = plan
            ctx.save_for_backward(u, c_points)
            return mf_apply(plan, c_points, u)

        @staticmethod
        def backward(ctx, gy):
            u, c_points = ctx.saved_tensors
            du, dc = mf_adjoint(ctx.plan, c_points, u, gy.contiguous())
            return du, dc, None

    return MassApply


_MassApply = None


def mass_apply(u, c_points, plan):
    """Differentiable y = M(c) u (autograd through the hand-written adjoint)."""
    global _MassApply
    if _MassApply is None:
        _MassApply = _make_mass_apply()
    return _MassApply.apply(u, c_points, plan)


class Batch:
    """Batched formation of several set-up plans (one persistent launch, optional HIP graph).

    The plans, coefficients and output tensors are kept referenced: the
    library borrows them for the batch's life.
    """

    def __init__(self, plans, coeffs=None, outs=None):
        torch = _torch()
        self.plans = list(plans)
        self.coeffs = [p.coeff() for p in self.plans] if coeffs is None else list(coeffs)
        self.outs = outs if outs is not None else [
            torch.empty((p.sizes["band"], p.sizes["n_act"]), dtype=torch.float64, device="cuda") for p in self.plans]
        n = len(self.plans)
        hs = (C.c_void_p * n)(*[p.h for p in self.plans])
        cs = (iga_coeff * n)(*self.coeffs)
        vs = (C.c_void_p * n)(*[_dptr(o) for o in self.outs])
        self.h = C.c_void_p()
        _check(lib().iga_batch_create(hs, n, cs, vs, C.byref(self.h)))

    def form(self, use_graph=False, stream=None):
        _check(lib().iga_batch_form(self.h, 1 if use_graph else 0, _stream(stream)))
        return self.outs

    def autotune(self, stream=None):
        ms = C.c_float()
        _check(lib().iga_batch_autotune(self.h, _stream(stream), C.byref(ms)))
        return ms.value

    def info(self):
        st = iga_batch_stats()
        _check(lib().iga_batch_info(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def status(self, stream=None):
        _check(lib().iga_batch_status(self.h, _stream(stream)))

    def project(self, targets, rtol=1e-12, maxit=None, u0=None, stream=None, raise_on_noconv=True):
        """Batched L2 projection of every patch (after form); returns (list of u, list of info dicts)."""
        torch = _torch()
        n = len(self.plans)
        us = [torch.zeros(p.sizes["n_act"], dtype=torch.float64, device="cuda") if u0 is None else u0[k].clone()
              for k, p in enumerate(self.plans)]
        gs = (iga_target * n)(*targets)
        up = (C.c_void_p * n)(*[_dptr(u) for u in us])
        infos = (iga_solve_info * n)()
        maxit = maxit or 10 * max(p.sizes["n_act"] for p in self.plans)
        code = lib().iga_batch_project(self.h, gs, rtol, maxit, up, infos, _stream(stream))
        out = [{"iterations": i.iterations, "converged": bool(i.converged), "rel_residual": i.rel_residual}
               for i in infos]
        if code != 0 and not (code == -8 and not raise_on_noconv):
            _check(code)
        return us, out

    def close(self):
        if getattr(self, "h", None):
            lib().iga_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mass_form_batched(plans, coeffs=None, outs=None, use_graph=False, stream=None):
    """One-shot batched formation (the C call builds, runs and frees a batch)."""
    torch = _torch()
    coeffs = [p.coeff() for p in plans] if coeffs is None else list(coeffs)
    outs = outs if outs is not None else [
        torch.empty((p.sizes["band"], p.sizes["n_act"]), dtype=torch.float64, device="cuda") for p in plans]
    n = len(plans)
    hs = (C.c_void_p * n)(*[p.h for p in plans])
    cs = (iga_coeff * n)(*coeffs)
    vs = (C.c_void_p * n)(*[_dptr(o) for o in outs])
    _check(lib().iga_trim_mass_form_batched(hs, n, cs, vs, 1 if use_graph else 0, _stream(stream)))
    return outs
