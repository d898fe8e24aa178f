// C ABI of the library (declared in include/iga_trim.h): plan creation,
// formation, status, timing. Host code only orchestrates device work;
// every step of the method runs in the kernels of setup.hip, trim.hip,
// form.hip, solve.hip and matfree.hip.
#include <algorithm>
#include <memory>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"

namespace iga {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

Plan::~Plan() {
    if (fexec) hipGraphExecDestroy(fexec);
    if (fgraph) hipGraphDestroy(fgraph);
    if (cap_stream) hipStreamDestroy(cap_stream);
    if (sw.h_scal) hipHostFree(sw.h_scal);
    for (hipEvent_t e : {ev_fork, ev_iso, ev_lists, ev_interior, ev_band, ev_classes, ev_aux_lists})
        if (e) hipEventDestroy(e);
    if (aux) hipStreamDestroy(aux);
    for (auto& e : ev_pool) hipEventDestroy(e);
    for (void* ptr : allocations) hipFree(ptr);
}

// Readers of the index-check counts of the modules built with -DIGA_DEBUG_BOUNDS
// (each registers one at load time); none in a release build.
static std::vector<unsigned long long (*)(bool)>& bounds_readers() {
    static std::vector<unsigned long long (*)(bool)> v;
    return v;
}
int bounds_register(unsigned long long (*read)(bool reset)) {
    bounds_readers().push_back(read);
    return (int)bounds_readers().size();
}

static int qmax_of(int N, int p) {
    // most WQ points in the support of one function: elements i-p..i
    int best = 0;
    for (int i = 0; i < N + p; ++i) {
        int tot = 0;
        for (int e = std::max(0, i - p); e <= std::min(N - 1, i); ++e)
            tot += (e == 0 || e == N - 1) ? p + 1 : 2;
        best = std::max(best, tot);
    }
    return best;
}

template <typename T>
static void h2d(T* dst, const T* src, size_t n, hipStream_t s) {
    HIPX(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <typename T>
static T d2h1(const T* src, hipStream_t s) {
    T v;
    HIPX(hipMemcpyAsync(&v, src, sizeof(T), hipMemcpyDeviceToHost, s));
    HIPX(hipStreamSynchronize(s));
    return v;
}

// matfree.hip: device address of the allocation-free product's scratch array (once per device)
void mf_scratch_init(int device);
// dwq.hip: a DWQ plan's side rules as workgroups of the cut element matrices' launch
void launch_cut_elems_sides(Plan& P, const iga_coeff& c, hipStream_t s);
// dwq.hip: a DWQ plan's box parts into the plan's second row scratch array (added by the cut-entry launch)
void launch_dwq_box_parts(Plan& P, const iga_coeff& c, hipStream_t s);

static void check_status(Plan& P, hipStream_t s) {
    int st = d2h1(P.status, s);
    if (st != IGA_OK) {
        int z = 0;
        HIPX(hipMemcpyAsync(P.status, &z, sizeof(int), hipMemcpyHostToDevice, s));
        HIPX(hipStreamSynchronize(s));
        throw Error{st, st == IGA_E_SINGULAR_WEIGHTS ? "a weight system of Eq. (5) is rank deficient"
                                                     : "trimming geometry outside what is handled"};
    }
}

// Set-up kernels in dependency order. With `discover`, device counts are read
// back after each stage to size the next buffers (plan creation only).
// Univariate tables, weighted-quadrature weights (and DWQ side rules): they
// depend on the knots only.
static void setup_tables(Plan& P, hipStream_t s, bool sides = true) {
    launch_dir_tables(P, s);
    launch_wq_weights(P, s);
    if (sides) launch_dwq_sides(P, s);
}

// Trimming, classes, lists, cut rules and (with `points`) the grid and band
// entries of the rule-point table. The trimming reads the knots directly;
// only the rule points read the univariate tables.
// part 0: all of it; 1: up to the lists (and DWQ boxes), then ev_lists; 2: the cut rules and points;
// 3: up to the classes, then ev_classes (the lists then come from setup_lists on another stream).
static void setup_trim(Plan& P, hipStream_t s, bool discover, bool points, int part = 0);

// Compact maps, lists and DWQ boxes from the classes, then ev_lists.
static void setup_lists(Plan& P, hipStream_t s) {
    launch_trim_lists(P, s);
    launch_dwq_choose(P, s);
    HIPX(hipEventRecord(P.ev_lists, s));
}

static void run_setup(Plan& P, hipStream_t s, bool discover) {
    if (discover) launch_gauss_table(P, s);  // a constant table: once per plan
    setup_tables(P, s);
    setup_trim(P, s, discover, true);
}

static void setup_trim(Plan& P, hipStream_t s, bool discover, bool points, int part) {
    TrimDev& T = P.trim;
    if (part != 2) {
        if (T.n_curves > 0) {
            launch_trim_curves(P, s);
            if (discover) {  // one slot of arcs per piece, as many as the most crossings of a piece + 1
                T.arc_slot = trim_max_crossings(P, s) + 1;
                T.cap_arcs = std::max(T.cap_pieces, 1) * T.arc_slot;
                T.cross = P.alloc<CrossDev>(T.cap_arcs);
                T.merged = P.alloc<CrossDev>(T.cap_arcs);
                T.arcs = P.alloc<ArcDev>(T.cap_arcs);
                P.arc_next = P.alloc<int>(T.cap_arcs);
            }
            launch_trim_arcs(P, s);
        }
        launch_trim_classes(P, s);
        if (part == 3) {
            HIPX(hipEventRecord(P.ev_classes, s));
            return;
        }
        launch_trim_lists(P, s);
        if (discover) {
            int c[4];
            HIPX(hipMemcpyAsync(c, P.counts, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            P.n_act = c[0];
            P.n_form_rows = c[1];
            P.n_cut_el = c[2];
            P.n_band = c[3];
            int nc = (int)P.n_cut_el;
            P.cut_el = P.alloc<CutElemDev>(std::max(nc, 1));
            P.cut_e = P.alloc<int>(std::max(nc, 1));
            P.node_cnt = P.alloc<int>(nc + 1);
            P.node_off = P.alloc<int>(nc + 1);
            if (P.method == IGA_DWQ) P.dwq_region = P.alloc<int>(8 * (size_t)std::max<int64_t>(P.n_form_rows, 1));
        }
        launch_dwq_choose(P, s);
        HIPX(hipEventRecord(P.ev_lists, s));  // classes, compact maps and DWQ boxes are ready
    }
    if (part == 1) return;
    launch_trim_cutprep(P, s, !discover);  // after plan creation the cut rules' nodes are written with them
    if (discover) {
        // node offsets are formed with the nodes; their total is needed to size the buffers first
        P.n_nodes = 0;
        P.n_arcs = 0;
        if (P.n_cut_el > 0) {
            std::vector<int> cnt((size_t)P.n_cut_el);
            std::vector<CutElemDev> ce((size_t)P.n_cut_el);
            HIPX(hipMemcpyAsync(cnt.data(), P.node_cnt, cnt.size() * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPX(hipMemcpyAsync(ce.data(), P.cut_el, ce.size() * sizeof(CutElemDev), hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            for (int v : cnt) P.n_nodes += v;
            for (const CutElemDev& E : ce) P.n_arcs += E.narc;
        }
        size_t nn = std::max<int64_t>(P.n_nodes, 1);
        P.node_x = P.alloc<double>(nn);
        P.node_y = P.alloc<double>(nn);
        P.node_w = P.alloc<double>(nn);
        P.node_el = P.alloc<int>(nn);
        size_t L = (size_t)(P.p + 1) * (P.p + 1);
        P.cutE = P.alloc<double>(std::max<int64_t>(P.n_cut_el, 1) * L * L);
        // inside sums of the rows formed in two launches (and, for DWQ, their box parts after them)
        P.cut_part = P.alloc<double>((P.method == IGA_DWQ ? 2 : 1) * (size_t)std::max<int64_t>(P.n_form_rows, 1) *
                                     (2 * P.p + 1) * (2 * P.p + 1));
        size_t nq = (size_t)P.dir[0].Q * P.dir[1].Q;
        size_t nb = (size_t)P.n_band * L;
        P.n_points = (int64_t)(nq + nb + P.n_nodes);
        P.pts_xy = P.alloc<double>(2 * P.n_points);
        P.c_wq = P.alloc<double>(nq);
        P.c_band = P.alloc<double>(std::max<size_t>(nb, 1));
        P.c_cut = P.alloc<double>(nn);
        if (P.method == IGA_NAIVE_WQ) P.c_wq_masked = P.alloc<double>(nq);
    }
    if (discover) launch_trim_nodes(P, s);
    if (points) launch_points(P, s);
    if (discover) {
        check_status(P, s);
        int nf = P.n1 * P.n2;
        int* cnt = P.flags;
        int* out = P.flags + (nf + 1);
        launch_row_nnz(P, cnt, out, s);
        P.nnz = d2h1(out + P.n_act, s);
        // interior and cut counts
        std::vector<int8_t> fc(nf);
        HIPX(hipMemcpyAsync(fc.data(), P.fcls, nf, hipMemcpyDeviceToHost, s));
        HIPX(hipStreamSynchronize(s));
        P.n_interior = std::count(fc.begin(), fc.end(), (int8_t)FN_INTERIOR);
        P.n_cut_fn = std::count(fc.begin(), fc.end(), (int8_t)FN_CUT);
        if (P.method == IGA_DWQ && P.n_form_rows > 0) {
            std::vector<int> reg(8 * (size_t)P.n_form_rows);
            HIPX(hipMemcpyAsync(reg.data(), P.dwq_region, sizeof(int) * reg.size(), hipMemcpyDeviceToHost, s));
            HIPX(hipStreamSynchronize(s));
            P.n_dwq_rows = 0;
            for (int64_t r = 0; r < P.n_form_rows; ++r) P.n_dwq_rows += reg[8 * r] >= 0;
        }
    }
}

struct PhaseTimer {
    Plan& P;
    hipStream_t s;
    int phase;
    hipEvent_t a{}, b{};
    PhaseTimer(Plan& P_, hipStream_t s_, int ph) : P(P_), s(s_), phase(ph) {
        if (!P.timing) return;
        HIPX(hipEventCreate(&a));
        HIPX(hipEventCreate(&b));
        HIPX(hipEventRecord(a, s));
    }
    ~PhaseTimer() {
        if (!P.timing) return;
        hipEventRecord(b, s);
        P.ev_records.push_back({phase, {a, b}});
    }
};

// Naive weighted quadrature masks c with the trimming: formed on one stream.
static void form_serial(Plan& P, const iga_coeff& c, double* vals, int flags, hipStream_t s) {
    if (flags & IGA_FORM_FULL) {
        PhaseTimer t(P, s, IGA_PHASE_SETUP);
        run_setup(P, s, false);
    }
    {
        PhaseTimer t(P, s, IGA_PHASE_COEF);
        launch_coef(P, c, s);
        if (P.method == IGA_NAIVE_WQ) {
            const double* src = (c.kind == IGA_COEF_CONST) ? nullptr
                                : (c.kind == IGA_COEF_GEOM_DETJ ? P.c_wq : c.c_points);
            launch_naive_mask(P, src, c.value, s);
        }
    }
    {
        PhaseTimer t(P, s, IGA_PHASE_INTERIOR);
        launch_interior_rows(P, c, vals, s);
    }
    {
        PhaseTimer t(P, s, IGA_PHASE_CUT);
        launch_cut_rows(P, c, vals, s);
        launch_dwq_rows(P, c, vals, s);
    }
}

// Two streams: the caller's stream s carries the trimming chain, the cut
// rules, the band/cut coefficients and the cut rows; the plan's second
// stream carries the univariate tables and weights, the WQ-grid coefficient
// and the interior rows (after the compact maps exist); a DWQ plan's side
// rules run on s in the cut element matrices' launch.
// Both start after the work already queued on s and are joined back into s.
// Phase timers: SETUP and CUT on s, COEF (WQ grid) and INTERIOR on the second
// stream (they overlap).
static void form(Plan& P, const iga_coeff& c, double* vals, int flags, hipStream_t s) {
    if (P.method == IGA_NAIVE_WQ) {
        form_serial(P, c, vals, flags, s);
        return;
    }
    const bool full = (flags & IGA_FORM_FULL) != 0;
    const bool pts_by_coef = full && c.kind == IGA_COEF_GEOM_DETJ;  // the |det J| kernels write the rule points
    hipStream_t a = P.aux;
    // aux stream: univariate tables and weights, c on the WQ grid and the band
    // Gauss points, the inside sums of the rows formed element-wise, interior
    // rows, rule points; the caller's stream: trimming, classes, lists, cut
    // rules, cut element matrices (with c at the cut nodes) and their entries
    // in the rows formed element-wise.
    // Enqueued in the order the critical caller's stream needs them: the host
    // spends about as long enqueuing a formation as the device takes to run
    // it, so the trimming chain goes first, the cut rules right after the
    // auxiliary stream's first kernels.
    // With row offsets the list kernel sums itself, the cut rules find their
    // elements from the class kernel's counts, so the lists move to the
    // auxiliary stream, off the caller's (critical) one.
    const bool split = full && trim_lists_prefix_here(P);
    HIPX(hipEventRecord(P.ev_fork, s));
    if (full) {
        PhaseTimer t(P, s, IGA_PHASE_SETUP);
        setup_trim(P, s, false, false, split ? 3 : 1);
    } else {
        HIPX(hipEventRecord(P.ev_lists, s));
    }
    HIPX(hipStreamWaitEvent(a, P.ev_fork, 0));
    // A full DWQ formation runs the side rules (which read the knots only) on
    // the caller's stream, as workgroups of the cut element matrices' launch.
    if (full && c.kind == IGA_COEF_GEOM_DETJ) {
        // the weights and c on the WQ grid in one launch (the COEF phase times both)
        launch_dir_tables(P, a);
        PhaseTimer t(P, a, IGA_PHASE_COEF);
        launch_weights_coef(P, c, a, pts_by_coef);
    } else {
        if (full) setup_tables(P, a, false);
        PhaseTimer t(P, a, IGA_PHASE_COEF);
        launch_coef(P, c, a, 1, pts_by_coef);
    }
    if (full) {
        PhaseTimer t(P, s, IGA_PHASE_SETUP);
        setup_trim(P, s, false, false, 2);
    }
    if (split) {
        HIPX(hipStreamWaitEvent(a, P.ev_classes, 0));
        setup_lists(P, a);
    } else {
        HIPX(hipStreamWaitEvent(a, P.ev_lists, 0));
    }
    const bool box_early = P.method == IGA_DWQ && P.n_form_rows > 0;
    if (box_early) HIPX(hipEventRecord(P.ev_aux_lists, a));  // the box parts read c on the WQ grid and the boxes
    // The interior rows first (beside the cut rules, which leave most of the
    // GPU idle), then the inside sums of the element-formed rows (beside the
    // cut element matrices); the caller's stream joins once, before the cut
    // entries, which need those sums.
    if (P.timing) {
        // The interior kernel alone, events at its dispatch's start and end:
        // it waits for the work queued on s so far, and s waits for it before
        // its next kernel, so the events time the kernel and not its share
        // of a GPU busy with the cut rules.
        HIPX(hipEventRecord(P.ev_iso, s));
        HIPX(hipStreamWaitEvent(a, P.ev_iso, 0));
        hipEvent_t t0, t1;
        HIPX(hipEventCreate(&t0));
        HIPX(hipEventCreate(&t1));
        launch_interior_rows(P, c, vals, a, t0, t1);
        P.ev_records.push_back({IGA_PHASE_INTERIOR, {t0, t1}});
        HIPX(hipEventRecord(P.ev_interior, a));
        HIPX(hipStreamWaitEvent(s, P.ev_interior, 0));
    } else if (c.kind == IGA_COEF_GEOM_DETJ && P.method != IGA_GAUSS_REF && P.n_band > 0) {
        // the interior rows and c at the band Gauss points in one launch
        launch_interior_coef(P, c, vals, a, pts_by_coef);
    } else {
        launch_interior_rows(P, c, vals, a);
    }
    const bool band_coef_done = !P.timing && c.kind == IGA_COEF_GEOM_DETJ && P.method != IGA_GAUSS_REF && P.n_band > 0;
    if (full && !pts_by_coef) launch_points(P, a);
    {
        PhaseTimer t(P, a, IGA_PHASE_CUT);
        if (!band_coef_done) launch_coef(P, c, a, 3, pts_by_coef);
        launch_cut_rows_mode(P, c, vals, a, 1);  // rows formed element-wise: their inside sums
    }
    HIPX(hipEventRecord(P.ev_band, a));  // everything on the auxiliary stream is done
    {
        PhaseTimer t(P, s, IGA_PHASE_CUT);
        // DWQ up to degree 4: the side rules (from the knots alone) as workgroups of the cut element
        // matrices' launch; at degree 6 that launch's registers and LDS (the larger of the two bodies,
        // and both bodies' LDS) slow the cut element matrices more than the overlap saves
        if (full && P.method == IGA_DWQ && P.p <= 4) {
            launch_cut_elems_sides(P, c, s);
        } else {
            launch_cut_elems(P, c, s);  // with c at the cut nodes
            if (full) launch_dwq_sides(P, s);
        }
        if (box_early) {  // DWQ: the rows' box parts, while the second stream finishes
            HIPX(hipStreamWaitEvent(s, P.ev_aux_lists, 0));
            launch_dwq_box_parts(P, c, s);
        }
        HIPX(hipStreamWaitEvent(s, P.ev_band, 0));
        launch_cut_rows_mode(P, c, vals, s, 2);  // plus the cut element matrices' entries (and box parts)
    }
}

// The formation recorded once as a HIP graph and replayed: one submission
// instead of some forty kernel launches and stream joins. Kernel arguments
// are the plan's buffers and sizes, which stay fixed for its life, plus the
// output, the coefficient and the flags, which key the recording. The set-up
// counter that tags marks and lists lives on the device, so replays need no
// new argument.
static bool same_coeff(const iga_coeff& a, const iga_coeff& b) {
    return a.kind == b.kind && a.value == b.value && a.geom_cp == b.geom_cp && a.c_points == b.c_points;
}

static void form_graph(Plan& P, const iga_coeff& c, double* vals, int flags, hipStream_t s) {
    const bool recorded = P.fexec && P.fkey_vals == vals && P.fkey_flags == flags && same_coeff(P.fkey_c, c);
    if (!recorded && !(P.pkey_vals == vals && P.pkey_flags == flags && same_coeff(P.pkey_c, c))) {
        // a call unlike the last one runs kernel by kernel; a repeated one is recorded
        P.pkey_vals = vals;
        P.pkey_flags = flags;
        P.pkey_c = c;
        form(P, c, vals, flags, s);
        return;
    }
    if (!recorded) {
        if (P.fexec) HIPX(hipGraphExecDestroy(P.fexec));
        if (P.fgraph) HIPX(hipGraphDestroy(P.fgraph));
        P.fexec = nullptr;
        P.fgraph = nullptr;
        if (!P.cap_stream) HIPX(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
        HIPX(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeRelaxed));
        try {
            form(P, c, vals, flags, P.cap_stream);
        } catch (...) {
            hipGraph_t g = nullptr;
            hipStreamEndCapture(P.cap_stream, &g);
            if (g) hipGraphDestroy(g);
            throw;
        }
        HIPX(hipStreamEndCapture(P.cap_stream, &P.fgraph));
        HIPX(hipGraphInstantiate(&P.fexec, P.fgraph, nullptr, nullptr, 0));
        P.fkey_vals = vals;
        P.fkey_flags = flags;
        P.fkey_c = c;
    }
    HIPX(hipGraphLaunch(P.fexec, s));
}

static void validate_knots(const double* k, int n, int p, int d) {
    IGA_REQUIRE(k != nullptr && n >= 2 * p + 2, IGA_E_INVALID, "knot vector " + std::to_string(d) + " too short");
    for (int i = 0; i <= p; ++i) {
        IGA_REQUIRE(k[i] == 0.0, IGA_E_INVALID, "knot vectors must start with p+1 zeros");
        IGA_REQUIRE(k[n - 1 - i] == 1.0, IGA_E_INVALID, "knot vectors must end with p+1 ones");
    }
    for (int i = p; i < n - p - 1; ++i)
        IGA_REQUIRE(k[i + 1] > k[i], IGA_E_INVALID, "interior knots must be simple and increasing");
}

}  // namespace iga

using namespace iga;

#define API_BEGIN try {
#define API_END                               \
    }                                         \
    catch (const Error& e) {                  \
        set_error(e.msg);                     \
        return e.code;                        \
    }                                         \
    catch (const std::exception& e) {         \
        set_error(e.what());                  \
        return IGA_E_INVALID;                 \
    }                                         \
    return IGA_OK;

extern "C" {

int iga_trim_plan_create(const iga_patch_desc* desc, const iga_opts* opts, iga_plan** out) {
    API_BEGIN
    IGA_REQUIRE(desc && out, IGA_E_INVALID, "null argument");
    *out = nullptr;
    int p = desc->degree;
    IGA_REQUIRE(p >= 1 && p <= IGA_MAXP, IGA_E_UNSUPPORTED, "degree must be in 1..8");
    IGA_REQUIRE(desc->method >= IGA_GAUSS_REF && desc->method <= IGA_NAIVE_WQ, IGA_E_UNSUPPORTED, "unknown method");
    for (int d = 0; d < 2; ++d) validate_knots(desc->knots[d], desc->n_knots[d], p, d);
    IGA_REQUIRE(desc->n_curves >= 0 && (desc->n_curves == 0 || desc->curves), IGA_E_INVALID, "curves missing");
    bool all_ellipses = true;
    for (int c = 0; c < desc->n_curves; ++c) {
        const iga_curve& C = desc->curves[c];
        if (C.kind == IGA_CURVE_BSPLINE) {
            IGA_REQUIRE(C.degree >= 1 && C.degree <= 3, IGA_E_UNSUPPORTED, "curve degree must be 1..3");
            IGA_REQUIRE(C.n_cp > C.degree && C.cp, IGA_E_INVALID, "curve needs more control points than its degree");
            all_ellipses = false;
        } else if (C.kind == IGA_CURVE_ELLIPSE) {
            IGA_REQUIRE(C.a > 0 && C.b > 0, IGA_E_INVALID, "ellipse semi-axes must be positive");
        } else {
            throw Error{IGA_E_UNSUPPORTED, "unknown curve kind"};
        }
    }
    IGA_REQUIRE(desc->n_curves <= 1 || all_ellipses, IGA_E_UNSUPPORTED,
                "a union of several holes is handled for ellipses only");

    auto* P = new iga_plan();
    std::unique_ptr<iga_plan> guard(P);
    HIPX(hipGetDevice(&P->device));
    mf_scratch_init(P->device);  // the allocation-free product's scratch address on this device
    HIPX(hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking));
    for (hipEvent_t* e :
         {&P->ev_fork, &P->ev_iso, &P->ev_lists, &P->ev_interior, &P->ev_band, &P->ev_classes, &P->ev_aux_lists})
        HIPX(hipEventCreateWithFlags(e, hipEventDisableTiming));
    P->p = p;
    P->method = desc->method;

    if (opts)
        for (int k = 0; k < 5; ++k) IGA_REQUIRE(opts->reserved[k] == 0, IGA_E_INVALID, "reserved option fields must be 0");
    P->n_r = (opts && opts->n_r > 0) ? opts->n_r : p + 1;
    P->n_s = (opts && opts->n_s > 0) ? opts->n_s : p + 1;
    P->n_q_override = (opts && opts->n_q > 0) ? opts->n_q : 0;
    IGA_REQUIRE(P->n_r <= IGA_MAX_GAUSS && P->n_s <= IGA_MAX_GAUSS && P->n_q_override <= IGA_MAX_GAUSS &&
                    3 * (2 * p + 1) <= IGA_MAX_GAUSS,
                IGA_E_UNSUPPORTED, "rule sizes above 64 points");
    hipStream_t s;
    HIPX(hipStreamCreate(&s));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { hipStreamDestroy(s); }
    } sg{s};

    for (int d = 0; d < 2; ++d) {
        DirDev& D = P->dir[d];
        D.N = desc->n_knots[d] - 2 * p - 1;
        D.n = D.N + p;
        D.Q = (D.N == 1) ? p + 1 : 2 * D.N + 2 * p - 2;
        D.qmax = qmax_of(D.N, p);
        IGA_REQUIRE(D.qmax <= 64, IGA_E_UNSUPPORTED, "too many points in one support");
        P->h_knots[d].assign(desc->knots[d], desc->knots[d] + desc->n_knots[d]);
        P->knots[d] = P->alloc<double>(desc->n_knots[d]);
        h2d(P->knots[d], desc->knots[d], desc->n_knots[d], s);
        D.knots = P->knots[d];
        D.bp = P->alloc<double>(D.N + 1);
        D.xq = P->alloc<double>(D.Q);
        D.eq = P->alloc<int>(D.Q);
        D.pt0 = P->alloc<int>(D.N + 1);
        D.Bq = P->alloc<double>((size_t)D.Q * (p + 1));
        D.dBq = P->alloc<double>((size_t)D.Q * (p + 1));
        D.M1 = P->alloc<double>((size_t)D.n * (2 * p + 1));
        D.W = P->alloc<double>((size_t)D.n * D.qmax);
        D.WB = P->alloc<double>((size_t)D.n * D.qmax * (2 * p + 1));
        D.WBT = P->alloc<double>((size_t)D.n * (2 * p + 2) * (p + 1));
        D.WT = P->alloc<double>((size_t)D.n * (2 * p + 2));
        D.xg = P->alloc<double>((size_t)D.N * (p + 1));
        D.wg = P->alloc<double>((size_t)D.N * (p + 1));
        D.Bg = P->alloc<double>((size_t)D.N * (p + 1) * (p + 1));
        D.dBg = P->alloc<double>((size_t)D.N * (p + 1) * (p + 1));
        D.dq_KQ = 4 * p + 2;
        D.dq_n = nullptr;
        D.dq_x = nullptr;
        D.dq_el = nullptr;
        D.dq_k = nullptr;
        D.dq_w = nullptr;
        if (desc->method == IGA_DWQ && D.N > 1) {
            const size_t slots = 2 * (size_t)(D.N - 1);
            D.dq_n = P->alloc<int>(slots);
            D.dq_x = P->alloc<double>(slots * D.dq_KQ);
            D.dq_el = P->alloc<int>(slots * D.dq_KQ);
            D.dq_k = P->alloc<int>(slots * D.dq_KQ);
            D.dq_w = P->alloc<double>(slots * p * D.dq_KQ);
        }
    }
    P->N1 = P->dir[0].N;
    P->N2 = P->dir[1].N;
    P->n1 = P->dir[0].n;
    P->n2 = P->dir[1].n;
    P->gauss_x = P->alloc<double>(gauss_off(IGA_MAX_GAUSS + 1));
    P->gauss_w = P->alloc<double>(gauss_off(IGA_MAX_GAUSS + 1));
    P->status = P->alloc<int>(1);
    P->counts = P->alloc<int>(16);
    HIPX(hipMemsetAsync(P->status, 0, sizeof(int), s));

    // curves
    TrimDev& T = P->trim;
    T.n_curves = desc->n_curves;
    std::vector<double> cp;
    std::vector<int> cp_off;
    int nseg = 0;
    for (int c = 0; c < desc->n_curves; ++c) {
        const iga_curve& C = desc->curves[c];
        CurveDev D{};
        D.kind = C.kind;
        D.degree = C.degree;
        D.seg0 = nseg;
        D.cx = C.cx;
        D.cy = C.cy;
        D.a = C.a;
        D.b = C.b;
        D.phi = C.phi;
        D.sigma = 1.0;
        cp_off.push_back((int)(cp.size() / 2));
        if (C.kind == IGA_CURVE_BSPLINE) {
            D.n_seg = C.n_cp;
            D.t_range = 1.0;
            cp.insert(cp.end(), C.cp, C.cp + 2 * C.n_cp);
        } else {
            D.n_seg = 1;
            D.t_range = 2.0 * M_PI;
        }
        nseg += D.n_seg;
        P->h_curves.push_back(D);
    }
    T.n_segs = nseg;
    if (T.n_curves > 0) {
        IGA_REQUIRE(nseg <= 1 << 20, IGA_E_UNSUPPORTED, "too many curve segments");
        P->d_curves = P->alloc<CurveDev>(T.n_curves);
        h2d(P->d_curves, P->h_curves.data(), T.n_curves, s);
        T.curves = P->d_curves;
        P->d_cp = P->alloc<double>(std::max<size_t>(cp.size(), 2));
        if (!cp.empty()) h2d(P->d_cp, cp.data(), cp.size(), s);
        P->d_cp_off = P->alloc<int>(T.n_curves);
        h2d(P->d_cp_off, cp_off.data(), cp_off.size(), s);
        T.segs = P->alloc<SegDev>(nseg);
        T.cap_pieces0 = kMaxPiecesPerSeg * nseg;
        T.cap_pieces = (T.n_curves > 1) ? T.cap_pieces0 * (kMaxIsectPerPiece + 1) : T.cap_pieces0;
        T.pieces = P->alloc<PieceDev>(T.cap_pieces);
        T.pieces0 = (T.n_curves > 1) ? P->alloc<PieceDev>(T.cap_pieces0) : T.pieces;
        T.n_pieces = P->alloc<int>(1);
        T.n_pieces0 = (T.n_curves > 1) ? P->alloc<int>(1) : T.n_pieces;
        T.piece_curve_off = P->alloc<int>(T.n_curves + 1);
        T.isect_t = P->alloc<double>((size_t)T.cap_pieces0 * kMaxIsectPerPiece);
        T.isect_n = P->alloc<int>(T.cap_pieces0);
        T.row_cnt = P->alloc<int>(P->N2);
        T.row_key = P->alloc<double>((size_t)P->N2 * kRowCross);
        T.row_curve = P->alloc<int>((size_t)P->N2 * kRowCross);
    }
    int nf = P->n1 * P->n2, ne = P->N1 * P->N2;
    P->ecls = P->alloc<int8_t>(ne);
    P->emark = P->alloc<int>(ne);
    HIPX(hipMemsetAsync(P->emark, 0, sizeof(int) * (size_t)ne, s));
    P->d_epoch = P->alloc<int>(1);
    const int epoch0 = 1;  // above every mark's initial 0
    h2d(P->d_epoch, &epoch0, 1, s);
    HIPX(hipStreamSynchronize(s));
    T.epoch = P->d_epoch;
    P->ehead = P->alloc<unsigned long long>(ne);
    HIPX(hipMemsetAsync(P->ehead, 0, sizeof(unsigned long long) * (size_t)ne, s));
    P->cut_id = P->alloc<int>(ne);
    P->band_id = P->alloc<int>(ne);
    P->cut_list = P->alloc<int>(ne);
    P->band_list = P->alloc<int>(ne);
    P->fcls = P->alloc<int8_t>(nf);
    P->act_of = P->alloc<int>(nf);
    P->fn_of = P->alloc<int>(nf);
    P->form_rows = P->alloc<int>(nf);
    P->flags = P->alloc<int>(2 * (size_t)(nf + 1) + 2 * (size_t)(ne + 1));
    P->list_rcnt = P->alloc<int>(4 * (size_t)P->n2 * ((P->N1 + 15) / 16));
    int big = std::max(std::max(nf, ne), T.cap_pieces) + 2;
    P->scan_pos_off = ((big + 1023) / 1024 + 64 + 63) / 64 * 64;  // block sums first, then positions
    P->scan_tmp = P->alloc<int>((size_t)P->scan_pos_off + (size_t)big);

    run_setup(*P, s, true);
    HIPX(hipStreamSynchronize(s));
    *out = guard.release();
    API_END
}

void iga_plan_destroy(iga_plan* plan) {
    if (!plan) return;
    hipDeviceSynchronize();
    delete plan;
}

int iga_plan_sizes(const iga_plan* P, iga_sizes* s) {
    API_BEGIN
    IGA_REQUIRE(P && s, IGA_E_INVALID, "null argument");
    std::memset(s, 0, sizeof(*s));
    s->p = P->p;
    s->N1 = P->N1;
    s->N2 = P->N2;
    s->n1 = P->n1;
    s->n2 = P->n2;
    s->n_act = P->n_act;
    s->n_interior = P->n_interior;
    s->n_cut_fn = P->n_cut_fn;
    s->n_cut_el = P->n_cut_el;
    s->n_band_el = P->n_band;
    s->band = (int64_t)(2 * P->p + 1) * (2 * P->p + 1);
    s->q1 = P->dir[0].Q;
    s->q2 = P->dir[1].Q;
    s->n_cut_nodes = P->n_nodes;
    s->n_points = P->n_points;
    s->nnz = P->nnz;
    s->n_arcs = P->n_arcs;
    s->n_dwq_rows = P->n_dwq_rows;
    s->workspace_bytes = P->bytes;
    API_END
}

int iga_plan_points(const iga_plan* P, const double** xy, int64_t* npts) {
    API_BEGIN
    IGA_REQUIRE(P, IGA_E_INVALID, "null plan");
    if (xy) *xy = P->pts_xy;
    if (npts) *npts = P->n_points;
    API_END
}

int iga_plan_index_maps(const iga_plan* P, const int32_t** act_of, const int32_t** fn_of, const int8_t** fn_class) {
    API_BEGIN
    IGA_REQUIRE(P, IGA_E_INVALID, "null plan");
    if (act_of) *act_of = P->act_of;
    if (fn_of) *fn_of = P->fn_of;
    if (fn_class) *fn_class = P->fcls;
    API_END
}

int iga_trim_mass_form(iga_plan* P, const iga_coeff* c, double* vals, int32_t flags, void* stream) {
    API_BEGIN
    IGA_REQUIRE(P && c && vals, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(c->kind >= IGA_COEF_CONST && c->kind <= IGA_COEF_AT_POINTS, IGA_E_UNSUPPORTED, "coefficient kind");
    IGA_REQUIRE(c->kind != IGA_COEF_GEOM_DETJ || c->geom_cp, IGA_E_INVALID, "geometry control points missing");
    IGA_REQUIRE(c->kind != IGA_COEF_AT_POINTS || c->c_points, IGA_E_INVALID, "per-point coefficient missing");
    IGA_REQUIRE(!(P->method == IGA_DWQ && c->kind == IGA_COEF_AT_POINTS), IGA_E_UNSUPPORTED,
                "discontinuous weighted quadrature needs c at nested points: constant or |det J| only");
    hipStream_t s = (hipStream_t)stream;
    if (P->timing || P->ktiming || !P->use_graph || P->method == IGA_NAIVE_WQ) {
        form(*P, *c, vals, flags, s);
    } else {
        form_graph(*P, *c, vals, flags, s);
    }
    HIPX(hipGetLastError());
    API_END
}

int iga_plan_set_graph(iga_plan* P, int32_t enable) {
    API_BEGIN
    IGA_REQUIRE(P, IGA_E_INVALID, "null plan");
    P->use_graph = enable != 0;
    API_END
}

int iga_status_get(iga_plan* P, void* stream) {
    API_BEGIN
    IGA_REQUIRE(P, IGA_E_INVALID, "null plan");
    check_status(*P, (hipStream_t)stream);
    API_END
}

int iga_plan_set_timing(iga_plan* P, int32_t enable) {
    API_BEGIN
    IGA_REQUIRE(P, IGA_E_INVALID, "null plan");
    IGA_REQUIRE(enable >= 0 && enable <= 2, IGA_E_INVALID, "timing mode must be 0, 1 or 2");
    P->timing = enable == 1;
    P->ktiming = enable == 2;
    API_END
}

int iga_plan_kernel_times(iga_plan* P, iga_kernel_time* out, int32_t cap, int32_t* n_out) {
    API_BEGIN
    IGA_REQUIRE(P && n_out && (cap == 0 || out), IGA_E_INVALID, "null argument");
    std::vector<std::string> names;
    std::vector<double> ms;
    std::vector<int64_t> cnt;
    for (auto& r : P->k_records) {
        HIPX(hipEventSynchronize(r.b));
        float t = 0.f;
        HIPX(hipEventElapsedTime(&t, r.a, r.b));
        size_t k = 0;
        while (k < names.size() && names[k] != r.name) ++k;
        if (k == names.size()) {
            names.emplace_back(r.name);
            ms.push_back(0.0);
            cnt.push_back(0);
        }
        ms[k] += t;
        cnt[k] += 1;
        P->k_pool.push_back(r.a);
        P->k_pool.push_back(r.b);
    }
    P->k_records.clear();
    const int n = (int)names.size();
    for (int k = 0; k < n && k < cap; ++k) {
        std::snprintf(out[k].name, sizeof(out[k].name), "%s", names[k].c_str());
        out[k].ms = ms[k];
        out[k].count = cnt[k];
    }
    *n_out = n;
    API_END
}

int iga_plan_timings(iga_plan* P, double* ms, int64_t* counts) {
    API_BEGIN
    IGA_REQUIRE(P, IGA_E_INVALID, "null plan");
    for (auto& r : P->ev_records) {
        HIPX(hipEventSynchronize(r.second.second));
        float t = 0.f;
        HIPX(hipEventElapsedTime(&t, r.second.first, r.second.second));
        P->phase_ms[r.first] += t;
        P->phase_cnt[r.first] += 1;
        hipEventDestroy(r.second.first);
        hipEventDestroy(r.second.second);
    }
    P->ev_records.clear();
    for (int k = 0; k < IGA_PHASE_COUNT; ++k) {
        if (ms) ms[k] = P->phase_ms[k];
        if (counts) counts[k] = P->phase_cnt[k];
        P->phase_ms[k] = 0;
        P->phase_cnt[k] = 0;
    }
    API_END
}

int iga_plan_table(const iga_plan* P, int32_t table, int32_t dir, const double** ptr, int64_t* count,
                   int64_t* stride) {
    API_BEGIN
    IGA_REQUIRE(P && ptr, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(dir == 0 || dir == 1, IGA_E_INVALID, "direction must be 0 or 1");
    const DirDev& D = P->dir[dir];
    int64_t n = 0, st = 1;
    const double* p = nullptr;
    size_t L = (size_t)(P->p + 1) * (P->p + 1);
    switch (table) {
        case IGA_TABLE_WQ_POINTS: p = D.xq; n = D.Q; break;
        case IGA_TABLE_WQ_WEIGHTS: p = D.W; n = (int64_t)D.n * D.qmax; st = D.qmax; break;
        case IGA_TABLE_MASS_1D: p = D.M1; n = (int64_t)D.n * (2 * P->p + 1); st = 2 * P->p + 1; break;
        case IGA_TABLE_C_WQ: p = P->c_wq; n = (int64_t)P->dir[0].Q * P->dir[1].Q; break;
        case IGA_TABLE_C_BAND: p = P->c_band; n = P->n_band * (int64_t)L; break;
        case IGA_TABLE_C_CUT: p = P->c_cut; n = P->n_nodes; break;
        case IGA_TABLE_CUT_W: p = P->node_w; n = P->n_nodes; break;
        case IGA_TABLE_DWQ_X: p = D.dq_x; n = D.dq_x ? 2 * (int64_t)(D.N - 1) * D.dq_KQ : 0; st = D.dq_KQ; break;
        case IGA_TABLE_DWQ_W:
            p = D.dq_w;
            n = D.dq_w ? 2 * (int64_t)(D.N - 1) * P->p * D.dq_KQ : 0;
            st = D.dq_KQ;
            break;
        default: throw Error{IGA_E_INVALID, "unknown table"};
    }
    *ptr = p;
    if (count) *count = n;
    if (stride) *stride = st;
    API_END
}

int iga_plan_int_table(const iga_plan* P, int32_t table, int32_t dir, const int32_t** ptr, int64_t* count,
                       int64_t* stride) {
    API_BEGIN
    IGA_REQUIRE(P && ptr, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(dir == 0 || dir == 1, IGA_E_INVALID, "direction must be 0 or 1");
    const DirDev& D = P->dir[dir];
    const int64_t slots = D.dq_n ? 2 * (int64_t)(D.N - 1) : 0;
    int64_t n = 0, st = 1;
    const int* p = nullptr;
    switch (table) {
        case IGA_ITABLE_DWQ_NPTS: p = D.dq_n; n = slots; break;
        case IGA_ITABLE_DWQ_ELEM: p = D.dq_el; n = slots * D.dq_KQ; st = D.dq_KQ; break;
        case IGA_ITABLE_DWQ_WQIDX: p = D.dq_k; n = slots * D.dq_KQ; st = D.dq_KQ; break;
        case IGA_ITABLE_DWQ_BOX: p = P->dwq_region; n = P->dwq_region ? 8 * P->n_form_rows : 0; st = 8; break;
        case IGA_ITABLE_FORM_ROWS: p = P->form_rows; n = P->n_form_rows; break;
        default: throw Error{IGA_E_INVALID, "unknown table"};
    }
    *ptr = p;
    if (count) *count = n;
    if (stride) *stride = st;
    API_END
}

int iga_plan_set_weights(iga_plan* P, int32_t dir, const double* W, void* stream) {
    API_BEGIN
    IGA_REQUIRE(P && W, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(dir == 0 || dir == 1, IGA_E_INVALID, "direction must be 0 or 1");
    const DirDev& D = P->dir[dir];
    HIPX(hipMemcpyAsync(D.W, W, sizeof(double) * (size_t)D.n * D.qmax, hipMemcpyDefault, (hipStream_t)stream));
    launch_wb_table(*P, dir, (hipStream_t)stream);
    API_END
}

int iga_plan_set_dwq_weights(iga_plan* P, int32_t dir, const double* w, void* stream) {
    API_BEGIN
    IGA_REQUIRE(P && w, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(dir == 0 || dir == 1, IGA_E_INVALID, "direction must be 0 or 1");
    const DirDev& D = P->dir[dir];
    IGA_REQUIRE(P->method == IGA_DWQ, IGA_E_INVALID, "the plan's method is not IGA_DWQ");
    if (D.dq_w)
        HIPX(hipMemcpyAsync(D.dq_w, w, sizeof(double) * 2 * (size_t)(D.N - 1) * P->p * D.dq_KQ, hipMemcpyDefault,
                            (hipStream_t)stream));
    API_END
}

int iga_plan_set_cut_nodes(iga_plan* P, const double* x, const double* y, const double* w, int64_t n_in,
                           void* stream) {
    API_BEGIN
    IGA_REQUIRE(P && x && y && w, IGA_E_INVALID, "null argument");
    IGA_REQUIRE(n_in == P->n_nodes, IGA_E_INVALID,
                "node count " + std::to_string(n_in) + " differs from the plan's " + std::to_string(P->n_nodes));
    hipStream_t s = (hipStream_t)stream;
    size_t n = (size_t)P->n_nodes;
    if (n > 0) {
        HIPX(hipMemcpyAsync(P->node_x, x, n * sizeof(double), hipMemcpyDefault, s));
        HIPX(hipMemcpyAsync(P->node_y, y, n * sizeof(double), hipMemcpyDefault, s));
        HIPX(hipMemcpyAsync(P->node_w, w, n * sizeof(double), hipMemcpyDefault, s));
        launch_points(*P, s, true);
    }
    API_END
}

int iga_copy(void* dst, const void* src, int64_t bytes, void* stream) {
    API_BEGIN
    IGA_REQUIRE(bytes >= 0 && (bytes == 0 || (dst && src)), IGA_E_INVALID, "bad copy arguments");
    if (bytes > 0) {
        HIPX(hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDefault, (hipStream_t)stream));
        HIPX(hipStreamSynchronize((hipStream_t)stream));
    }
    API_END
}

int iga_debug_bounds_hits(int64_t* hits, int32_t reset) {
    API_BEGIN
    IGA_REQUIRE(hits, IGA_E_INVALID, "null argument");
    *hits = 0;
#ifdef IGA_DEBUG_BOUNDS
    HIPX(hipDeviceSynchronize());
    unsigned long long total = 0;
    for (auto read : bounds_readers()) {
        const unsigned long long v = read(reset != 0);
        IGA_REQUIRE(v != ~0ull, IGA_E_HIP, "reading an index-check count failed");
        total += v;
    }
    *hits = (int64_t)total;
#else
    (void)reset;
    throw Error{IGA_E_UNSUPPORTED, "index checks are compiled in with -DIGA_DEBUG_BOUNDS only"};
#endif
    API_END
}

const char* iga_status_string(int code) {
    switch (code) {
        case IGA_OK: return "ok";
        case IGA_E_INVALID: return "invalid argument";
        case IGA_E_UNSUPPORTED: return "unsupported";
        case IGA_E_NOMEM: return "out of device memory";
        case IGA_E_HIP: return "HIP runtime error";
        case IGA_E_SINGULAR_WEIGHTS: return "singular weight system";
        case IGA_E_TOPOLOGY: return "unsupported trimming topology";
        case IGA_E_CAPACITY: return "capacity exceeded";
        case IGA_E_NOCONV: return "no convergence";
        default: return "unknown status";
    }
}

const char* iga_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
