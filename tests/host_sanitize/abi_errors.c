/* Error paths of every C-ABI call, for a host build of the library with
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only: the
 * device code is not compiled in, and no kernel is launched).
 *
 * Each call is made with arguments the header documents as invalid (null
 * plans and buffers, out-of-range degrees, methods and kinds, knot vectors
 * that are not open or not simple, malformed curves) and must return the
 * documented negative status with a message from iga_last_error(); a valid
 * descriptor must fail cleanly when no device can take the plan (the
 * library's clean-up path on a partly built plan). The sanitizers report
 * any invalid memory access, leak-free clean-up aside, or undefined
 * behaviour along the way; the program exits non-zero on the first failed
 * check. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "iga_trim.h"

static int failures = 0;

static void expect(const char* what, int got, int want) {
    const char* msg = iga_last_error();
    if (got != want || msg == NULL || (want != IGA_OK && msg[0] == '\0')) {
        fprintf(stderr, "FAIL %s: status %d (want %d), message \"%s\"\n", what, got, want, msg ? msg : "(null)");
        ++failures;
    } else {
        printf("ok   %-48s %d  %s\n", what, got, msg);
    }
}

static void expect_negative(const char* what, int got) {
    const char* msg = iga_last_error();
    if (got >= 0 || msg == NULL || msg[0] == '\0') {
        fprintf(stderr, "FAIL %s: status %d, message \"%s\"\n", what, got, msg ? msg : "(null)");
        ++failures;
    } else {
        printf("ok   %-48s %d  %s\n", what, got, msg);
    }
}

/* open uniform knot vector of N elements, degree p */
static double* open_knots(int N, int p, int* n) {
    *n = N + 2 * p + 1;
    double* k = (double*)malloc(sizeof(double) * (size_t)*n);
    for (int i = 0; i < *n; ++i) {
        const int j = i - p;
        k[i] = j <= 0 ? 0.0 : (j >= N ? 1.0 : (double)j / N);
    }
    return k;
}

static iga_patch_desc circle_desc(const double* k1, int n1, const double* k2, int n2, const iga_curve* cv, int p) {
    iga_patch_desc d;
    memset(&d, 0, sizeof d);
    d.degree = p;
    d.method = IGA_HYBRID_GAUSS;
    d.n_knots[0] = n1;
    d.n_knots[1] = n2;
    d.knots[0] = k1;
    d.knots[1] = k2;
    d.n_curves = 1;
    d.curves = cv;
    return d;
}

int main(void) {
    /* status strings */
    for (int code = -10; code <= 1; ++code) {
        const char* s = iga_status_string(code);
        if (s == NULL || s[0] == '\0') {
            fprintf(stderr, "FAIL iga_status_string(%d)\n", code);
            ++failures;
        }
    }

    const int p = 2, N = 8;
    int nk = 0;
    double* k = open_knots(N, p, &nk);
    iga_curve circle;
    memset(&circle, 0, sizeof circle);
    circle.kind = IGA_CURVE_ELLIPSE;
    circle.cx = 0.5;
    circle.cy = 0.5;
    circle.a = circle.b = 0.25;
    iga_plan* plan = (iga_plan*)0x1;  /* must be reset to NULL by the failing call */

    /* ---- plan creation: descriptor checks */
    iga_patch_desc d = circle_desc(k, nk, k, nk, &circle, p);
    expect("create: null descriptor", iga_trim_plan_create(NULL, NULL, &plan), IGA_E_INVALID);
    expect("create: null out", iga_trim_plan_create(&d, NULL, NULL), IGA_E_INVALID);
    d.degree = 0;
    expect("create: degree 0", iga_trim_plan_create(&d, NULL, &plan), IGA_E_UNSUPPORTED);
    d.degree = 9; /* the header allows 1..8 */
    expect("create: degree above the maximum", iga_trim_plan_create(&d, NULL, &plan), IGA_E_UNSUPPORTED);
    d = circle_desc(k, nk, k, nk, &circle, p);
    d.method = 17;
    expect("create: unknown method", iga_trim_plan_create(&d, NULL, &plan), IGA_E_UNSUPPORTED);
    d = circle_desc(NULL, nk, k, nk, &circle, p);
    expect("create: null knots", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    d = circle_desc(k, 2 * p + 1, k, nk, &circle, p);
    expect("create: knot vector too short", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);

    double* bad = (double*)malloc(sizeof(double) * (size_t)nk);
    memcpy(bad, k, sizeof(double) * (size_t)nk);
    bad[0] = -0.5;
    d = circle_desc(k, nk, bad, nk, &circle, p);
    expect("create: knots not starting with p+1 zeros", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    memcpy(bad, k, sizeof(double) * (size_t)nk);
    bad[nk - 1] = 2.0;
    expect("create: knots not ending with p+1 ones", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    memcpy(bad, k, sizeof(double) * (size_t)nk);
    bad[p + 2] = bad[p + 1];
    expect("create: repeated interior knot", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    memcpy(bad, k, sizeof(double) * (size_t)nk);
    bad[p + 2] = 0.5 * bad[p + 1];
    expect("create: decreasing interior knots", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);

    d = circle_desc(k, nk, k, nk, NULL, p);
    expect("create: curves missing", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    d = circle_desc(k, nk, k, nk, &circle, p);
    d.n_curves = -1;
    expect("create: negative curve count", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);

    const double cp[8] = {0.3, 0.3, 0.7, 0.3, 0.7, 0.7, 0.3, 0.7};
    iga_curve spl;
    memset(&spl, 0, sizeof spl);
    spl.kind = IGA_CURVE_BSPLINE;
    spl.degree = 4;
    spl.n_cp = 4;
    spl.cp = cp;
    d = circle_desc(k, nk, k, nk, &spl, p);
    expect("create: curve degree 4", iga_trim_plan_create(&d, NULL, &plan), IGA_E_UNSUPPORTED);
    spl.degree = 3;
    spl.n_cp = 3;
    expect("create: too few control points", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    spl.n_cp = 4;
    spl.cp = NULL;
    expect("create: control points missing", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    spl.cp = cp;
    iga_curve two[2] = {spl, spl};
    d.curves = two;
    d.n_curves = 2;
    expect("create: two B-spline holes", iga_trim_plan_create(&d, NULL, &plan), IGA_E_UNSUPPORTED);
    iga_curve flat = circle;
    flat.b = 0.0;
    d = circle_desc(k, nk, k, nk, &flat, p);
    expect("create: ellipse with a zero semi-axis", iga_trim_plan_create(&d, NULL, &plan), IGA_E_INVALID);
    iga_curve odd = circle;
    odd.kind = 9;
    d = circle_desc(k, nk, k, nk, &odd, p);
    expect("create: unknown curve kind", iga_trim_plan_create(&d, NULL, &plan), IGA_E_UNSUPPORTED);
    if (plan != NULL) {
        fprintf(stderr, "FAIL: a failed creation left *out set\n");
        ++failures;
    }

    /* a valid descriptor: no device (or no device code) can take it, so the
     * creation fails after its argument checks and frees what it built */
    d = circle_desc(k, nk, k, nk, &circle, p);
    iga_opts o;
    memset(&o, 0, sizeof o);
    plan = (iga_plan*)0x1;
    expect_negative("create: valid patch without a device", iga_trim_plan_create(&d, &o, &plan));
    if (plan != NULL) {
        fprintf(stderr, "FAIL: a failed creation left *out set\n");
        ++failures;
    }

    /* ---- every call on a null plan or batch */
    iga_sizes sz;
    iga_coeff c;
    memset(&c, 0, sizeof c);
    iga_target g;
    memset(&g, 0, sizeof g);
    iga_solve_info info;
    double buf[4] = {0, 0, 0, 0};
    const double* dp = NULL;
    const int32_t* ip = NULL;
    const int8_t* cp8 = NULL;
    int64_t cnt = 0, stride = 0;
    int32_t n32 = 0;
    float ms = 0.f;
    double phase_ms[IGA_PHASE_COUNT];
    int64_t phase_n[IGA_PHASE_COUNT];
    iga_kernel_time kt[2];
    iga_batch* batch = (iga_batch*)0x1;
    iga_batch_stats bst;
    iga_peaks pk;

    iga_plan_destroy(NULL);
    iga_batch_destroy(NULL);
    expect("sizes", iga_plan_sizes(NULL, &sz), IGA_E_INVALID);
    expect("points", iga_plan_points(NULL, &dp, &cnt), IGA_E_INVALID);
    expect("index maps", iga_plan_index_maps(NULL, &ip, &ip, &cp8), IGA_E_INVALID);
    expect("mass form", iga_trim_mass_form(NULL, &c, buf, IGA_FORM_FULL, NULL), IGA_E_INVALID);
    expect("set graph", iga_plan_set_graph(NULL, 1), IGA_E_INVALID);
    expect("status", iga_status_get(NULL, NULL), IGA_E_INVALID);
    expect("l2 project", iga_trim_l2_project(NULL, &c, buf, &g, 1e-12, 10, buf, &info, NULL), IGA_E_INVALID);
    expect("rhs", iga_trim_rhs(NULL, &c, &g, buf, NULL), IGA_E_INVALID);
    expect("l2 project (extended)", iga_trim_l2_project_ext(NULL, &c, buf, &g, 1e-12, 10, buf, &info, NULL),
           IGA_E_INVALID);
    expect("extension", iga_trim_extension(NULL, &n32, buf, NULL), IGA_E_INVALID);
    expect("matrix-free product", iga_mf_apply(NULL, buf, buf, buf, NULL), IGA_E_INVALID);
    expect("matrix-free product (no allocation)", iga_mf_apply_noalloc(NULL, buf, buf, buf, NULL), IGA_E_INVALID);
    expect("matrix-free adjoint", iga_mf_adjoint(NULL, buf, buf, buf, buf, buf, NULL), IGA_E_INVALID);
    expect("set timing", iga_plan_set_timing(NULL, 1), IGA_E_INVALID);
    expect("timings", iga_plan_timings(NULL, phase_ms, phase_n), IGA_E_INVALID);
    expect("kernel times", iga_plan_kernel_times(NULL, kt, 2, &n32), IGA_E_INVALID);
    expect("table", iga_plan_table(NULL, IGA_TABLE_WQ_POINTS, 0, &dp, &cnt, &stride), IGA_E_INVALID);
    expect("int table", iga_plan_int_table(NULL, IGA_ITABLE_FORM_ROWS, 0, &ip, &cnt, &stride), IGA_E_INVALID);
    expect("set weights", iga_plan_set_weights(NULL, 0, buf, NULL), IGA_E_INVALID);
    expect("set DWQ weights", iga_plan_set_dwq_weights(NULL, 0, buf, NULL), IGA_E_INVALID);
    expect("set cut nodes", iga_plan_set_cut_nodes(NULL, buf, buf, buf, 1, NULL), IGA_E_INVALID);
    expect("copy", iga_copy(NULL, NULL, -1, NULL), IGA_E_INVALID);
    expect("measure peaks", iga_measure_peaks(NULL, NULL, 0, 1, &pk, NULL), IGA_E_INVALID);

    iga_plan* plans[2] = {NULL, NULL};
    double* outs[2] = {buf, buf};
    iga_coeff cs[2] = {c, c};
    expect("batch create: no plans", iga_batch_create(NULL, 1, cs, outs, &batch), IGA_E_INVALID);
    expect("batch create: count 0", iga_batch_create(plans, 0, cs, outs, &batch), IGA_E_INVALID);
    expect("batch create: null plan", iga_batch_create(plans, 2, cs, outs, &batch), IGA_E_INVALID);
    if (batch != NULL) {
        fprintf(stderr, "FAIL: a failed batch creation left *out set\n");
        ++failures;
    }
    expect("batch form", iga_batch_form(NULL, 1, NULL), IGA_E_INVALID);
    expect("batch autotune", iga_batch_autotune(NULL, NULL, &ms), IGA_E_INVALID);
    expect("batch info", iga_batch_info(NULL, &bst), IGA_E_INVALID);
    expect("batch status", iga_batch_status(NULL, NULL), IGA_E_INVALID);
    double* us[2] = {buf, buf};
    expect("batch project", iga_batch_project(NULL, &g, 1e-12, 10, us, &info, NULL), IGA_E_INVALID);
    expect("batched form: null plan", iga_trim_mass_form_batched(plans, 2, cs, outs, 1, NULL), IGA_E_INVALID);

    free(bad);
    free(k);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("all checks passed\n");
    return 0;
}
